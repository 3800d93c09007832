"""The boundary without Python: tests/helpers/abi_client.c, a plain C99
program that links librwmi.so and lets the library allocate its own device
memory and stream, runs an FP64 domain (a sliding wall, a body force, a
metaball on a sinusoidal path, uniform walkers) and prints its moments,
velocity sums and occupancy.  The same domain built through the Python
binding (device memory from PyTorch's allocator, a PyTorch stream) must
give the same values bit for bit, with either fluid-particle coupling."""
import os
import subprocess
import sys

import numpy as np
import pytest

from test_abi import build_c_client

pytestmark = pytest.mark.gpu

STEPS = 40


def _binding_run(coupling):
    from paper_2308_05007_amd import binding as B
    dom = {"n": (20, 14, 24), "bc": ("periodic", "wall", "periodic"),
           "wall_hi": [[0.0, 0.0, 0.0], [0.01, 0.0, 0.0], [0.0, 0.0, 0.0]],
           "tau": 0.8, "F": (1e-5, 0.0, 0.0), "D": 0.02, "rho0": 1.0, "seed": 0x1234567890abcdef,
           "precision": "fp64"}
    d = B.Domain(dom)
    d.add_particle({"b": np.array([[-0.8, 0.0, 0.0], [0.8, 0.3, 0.0]]), "k": np.array([0.6, 0.5]),
                    "centre": (10.0, 7.0, 12.0), "motion": "sinusoid", "amp": (1.5, 0.0, 0.5), "period": 30.0,
                    "phase": 0.1})
    if coupling:
        d.set_fluid_coupling("ibb")
    seeded = d.seed({"kind": "uniform", "ref": (10.0, 7.0, 12.0), "sigma": 1.0, "band": (2, 0.0, 1.0),
                     "max_attempts": 64}, 3000)
    d.step(STEPS)
    d.sync()
    m = d.moments()
    u, _ = d.velocity()
    occ = d.occupancy()
    out = {"seeded": seeded, "step": m["step"], "n_walkers": m["n_walkers"], "mass": m["mass"],
           "type2": m["counters"]["type2"], "type4": m["counters"]["type4"],
           "wall_reflect": m["counters"]["wall_reflect"],
           "returned_to_origin": m["counters"]["returned_to_origin"], "occupancy": int(occ.sum())}
    for a in range(3):
        out["sum%d" % a] = m["sum"][a]
        out["sumsq%d" % a] = m["sumsq"][a]
        out["fluid_u%d" % a] = m["fluid_u"][a]
        s = 0.0
        for v in u[a].ravel().tolist():  # the client's order: one node after another
            s += v
        out["usum%d" % a] = s
    d.close()
    return out


def _client_run(exe, coupling):
    print("abi_client: %d steps, coupling %d" % (STEPS, coupling), flush=True)
    r = subprocess.run([exe, str(STEPS), str(coupling)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        k, v = line.split()
        out[k] = float.fromhex(v) if ("p" in v or "." in v) else int(v)
    return out


@pytest.mark.parametrize("coupling", [0, 1], ids=["psm", "ibb"])
def test_c_client_equals_binding(tmp_path, coupling):
    exe = build_c_client(tmp_path)
    got = _client_run(exe, coupling)
    ref = _binding_run(coupling)
    assert got["seeded"] == 3000 and got["n_walkers"] == 3000 and got["occupancy"] == 3000
    assert got["step"] == STEPS
    assert set(got) == set(ref), set(got) ^ set(ref)
    for k, v in ref.items():
        assert got[k] == v, (k, got[k], v)
