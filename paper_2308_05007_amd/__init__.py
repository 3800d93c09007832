"""MI355X-native hot path of RW-MI-DELBM (arXiv 2308.05007).

The compiled library (``librwmi.so``, HIP for gfx950) does all the work; this
package only marshals arguments (``binding``) and holds the seeded input
generators (``workloads``), the batch autotuner and the serving loop.  Importing
the package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
