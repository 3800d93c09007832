"""ctypes binding of librwmi (include/rwmi.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch, when
present with a GPU, supplies device memory (its caching allocator, through
the library's allocation callbacks) and the stream each domain runs on.
Loading fails loudly if librwmi.so has not been built: there is no CPU path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librwmi.so")

RWMI_OK, RWMI_EINVAL, RWMI_ENOMEM, RWMI_EDEVICE, RWMI_ESTATE, RWMI_ESEED = 0, -1, -2, -3, -4, -5
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ESEED"}
PRECISION = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
MOTION = {"static": 0, "sinusoid": 1, "const_vel": 2, "coupled": 3}
SEED_KIND = {"uniform": 0, "gaussian": 1, "band": 2, "explicit": 3}
KEY = {"max_bisect": 1, "use_graph": 2, "block": 3, "timing": 5, "step_flags": 6, "sort_every": 7, "streaming": 8, "member_blocks": 10}
MAX_PARTICLES = 64

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class DomainDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("wall_u_lo", (C.c_double * 3) * 3),
                ("wall_u_hi", (C.c_double * 3) * 3), ("tau", C.c_double), ("force", C.c_double * 3),
                ("diffusivity", C.c_double), ("rho0", C.c_double), ("u0", C.c_double * 3), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class MetaballDesc(C.Structure):
    _fields_ = [("n_ctrl", C.c_int32), ("offsets", C.POINTER(C.c_double)), ("weights", C.POINTER(C.c_double)),
                ("centre", C.c_double * 3), ("motion", C.c_int32), ("amplitude", C.c_double * 3),
                ("period", C.c_double), ("phase", C.c_double), ("velocity", C.c_double * 3)]


class SeedDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("centre", C.c_double * 3), ("sigma", C.c_double), ("band_axis", C.c_int32),
                ("band_lo", C.c_double), ("band_hi", C.c_double), ("xyz", C.POINTER(C.c_double)),
                ("ref", C.c_double * 3), ("max_attempts", C.c_int32), ("remove_inside", C.c_int32)]


class CouplingDesc(C.Structure):
    _fields_ = [("density", C.c_double), ("gravity", C.c_double * 3), ("drive_amplitude", C.c_double),
                ("drive_period", C.c_double), ("drive_direction", C.c_double * 3), ("kn", C.c_double),
                ("kt", C.c_double), ("eta_n", C.c_double), ("eta_t", C.c_double), ("mu", C.c_double),
                ("dilation_radius", C.c_double), ("substeps", C.c_int32), ("coupling", C.c_int32)]


# coupling parameters by the names of the particle dynamics (Eq. 4-11)
COUPLING_DEFAULTS = {"g": (0.0, 0.0, 0.0), "drive_amp": 0.0, "drive_period": 5000.0, "drive_dir": (1.0, 0.0, 0.0),
                     "kt": 0.0, "eta_n": 0.0, "eta_t": 0.0, "mu": 0.0, "nsub": 100, "coupling": 1}


def coupling_desc(dem):
    v = dict(COUPLING_DEFAULTS, **dem)
    c = CouplingDesc()
    c.density = float(v["rho_p"])
    for a in range(3):
        c.gravity[a] = float(v["g"][a])
        c.drive_direction[a] = float(v["drive_dir"][a])
    c.drive_amplitude = float(v["drive_amp"])
    c.drive_period = float(v["drive_period"])
    c.kn, c.kt = float(v["kn"]), float(v["kt"])
    c.eta_n, c.eta_t = float(v["eta_n"]), float(v["eta_t"])
    c.mu = float(v["mu"])
    c.dilation_radius = float(v["Rs"])
    c.substeps = int(v["nsub"])
    c.coupling = int(v["coupling"])
    return c


class Dispersion(C.Structure):
    _fields_ = [("u_slip", C.c_double), ("phi", C.c_double), ("K", C.c_double), ("D_alpha", C.c_double),
                ("offset", C.c_double)]


class Moments(C.Structure):
    _fields_ = [("step", C.c_uint64), ("n_walkers", C.c_uint64), ("sum", C.c_double * 3), ("sumsq", C.c_double * 3),
                ("mass", C.c_double), ("momentum", C.c_double * 3), ("fluid_u", C.c_double * 3),
                ("particle_v", C.c_double * 3), ("solid_volume", C.c_double), ("type2", C.c_uint64),
                ("type4", C.c_uint64), ("bisect_fail", C.c_uint64), ("refill_fallback", C.c_uint64),
                ("returned_to_origin", C.c_uint64), ("wall_reflect", C.c_uint64), ("near_surface", C.c_uint64),
                ("contact_misses", C.c_uint64)]


# name -> (restype, argtypes); the full exported surface of include/rwmi.h
SIGNATURES = {
    "rwmi_create_domain": (C.c_int, [C.POINTER(DomainDesc), C.POINTER(C.c_void_p)]),
    "rwmi_destroy_domain": (None, [C.c_void_p]),
    "rwmi_add_metaball_particle": (C.c_int, [C.c_void_p, C.POINTER(MetaballDesc), C.POINTER(C.c_int32)]),
    "rwmi_set_coupling": (C.c_int, [C.c_void_p, C.POINTER(CouplingDesc)]),
    "rwmi_set_fluid_coupling": (C.c_int, [C.c_void_p, C.c_int32]),
    "rwmi_read_particle_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "rwmi_set_particle_motion": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "rwmi_seed_walkers": (C.c_int, [C.c_void_p, C.POINTER(SeedDesc), C.c_uint64, C.POINTER(C.c_uint64)]),
    "rwmi_step": (C.c_int, [C.c_void_p, C.c_uint32]),
    "rwmi_read_moments": (C.c_int, [C.c_void_p, C.POINTER(Moments)]),
    "rwmi_read_moments_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Moments)]),
    "rwmi_read_occupancy": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rwmi_read_profile": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "rwmi_read_velocity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "rwmi_read_walkers": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rwmi_read_distributions": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rwmi_query_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "rwmi_footprint_bytes": (C.c_uint64, [C.POINTER(DomainDesc), C.c_uint32, C.c_uint32, C.c_uint64]),
    "rwmi_debug_set": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64]),
    "rwmi_read_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "rwmi_read_coupling_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                           C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "rwmi_synchronize": (C.c_int, [C.c_void_p]),
    "rwmi_last_error": (C.c_char_p, [C.c_void_p]),
    "rwmi_batch_create": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "rwmi_batch_add": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rwmi_batch_remove": (C.c_int, [C.c_void_p, C.c_void_p]),
    "rwmi_batch_step": (C.c_int, [C.c_void_p, C.c_uint32]),
    "rwmi_batch_set": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64]),
    "rwmi_batch_synchronize": (C.c_int, [C.c_void_p]),
    "rwmi_batch_destroy": (None, [C.c_void_p]),
    "rwmi_dispersion_from_moments": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32,
                                               C.c_uint64, C.c_double, C.c_void_p, C.c_void_p]),
    "rwmi_gaussian_fit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rwmi_device_normals": (C.c_int, [C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p]),
    "rwmi_stream_probe": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "rwmi_dispersion_fit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_double, C.c_double,
                                      C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
}

_lib = None


class RwmiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process."""
    try:
        with open("/proc/self/maps") as fh:
            return sorted({ln.split()[-1] for ln in fh if "libamdhip64" in ln and "/" in ln})
    except OSError:
        return []


def lib():
    """Load librwmi.so (raises if it has not been built).

    torch (when installed) is imported first: it brings its own HIP runtime
    under the soname libamdhip64.so.7, and librwmi.so must bind to that same
    runtime rather than load a second one."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librwmi.so is not built (%s); run python -m paper_2308_05007_amd.build" % LIB_PATH)
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError("two HIP runtimes are loaded (%s); import torch before librwmi.so" % ", ".join(rts))
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st, handle=None):
    if st != RWMI_OK:
        msg = lib().rwmi_last_error(handle)
        raise RwmiError(st, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch_gpu():
    try:
        import torch
        return torch if torch.cuda.is_available() else None
    except Exception:
        return None


class _TorchAllocator:
    """Device memory from torch's caching allocator on a given stream."""

    def __init__(self, torch, device, stream):
        self.torch = torch
        self.device = device
        self.stream = stream

        def _alloc(nbytes, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
            except Exception:
                return None

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


def make_desc(dom, device=0, stream=None, allocator=None):
    d = DomainDesc()
    n = dom["n"]
    bc = dom.get("bc", ("periodic",) * 3)
    for a in range(3):
        d.n[a] = int(n[a])
        d.bc[a] = 1 if bc[a] in ("wall", 1) else 0
    wl = np.asarray(dom.get("wall_lo", np.zeros(9)), float).reshape(3, 3)
    wh = np.asarray(dom.get("wall_hi", np.zeros(9)), float).reshape(3, 3)
    for a in range(3):
        for c in range(3):
            d.wall_u_lo[a][c] = wl[a, c]
            d.wall_u_hi[a][c] = wh[a, c]
    d.tau = float(dom["tau"])
    F = dom.get("F", (0, 0, 0))
    u0 = dom.get("u0", (0, 0, 0))
    for a in range(3):
        d.force[a] = float(F[a])
        d.u0[a] = float(u0[a])
    d.diffusivity = float(dom.get("D", 0.0))
    d.rho0 = float(dom.get("rho0", 1.0))
    d.seed = int(dom.get("seed", 0)) & (2**64 - 1)
    d.precision = PRECISION[dom.get("precision", "fp64")]
    d.device = int(device)
    d.stream = stream
    if allocator is not None:
        d.alloc = allocator.alloc
        d.free = allocator.free
    return d


def footprint_bytes(dom, n_particles=0, n_ctrl_total=0, n_walkers=0):
    d = make_desc(dom)
    return int(lib().rwmi_footprint_bytes(C.byref(d), int(n_particles), int(n_ctrl_total), int(n_walkers)))


class Domain:
    """One simulation domain on the GPU (mirrors the C ABI)."""

    def __init__(self, dom, device=0, use_torch=True):
        L = lib()
        self.L = L
        self.n = tuple(int(v) for v in dom["n"])
        self.N = int(np.prod(self.n))
        self.precision = dom.get("precision", "fp64")
        torch = _torch_gpu() if use_torch else None
        self._torch_stream = None
        self._alloc = None
        stream = None
        if torch is not None:
            self._torch_stream = torch.cuda.Stream(device=device)
            stream = C.c_void_p(self._torch_stream.cuda_stream)
            self._alloc = _TorchAllocator(torch, device, self._torch_stream.cuda_stream)
        self._desc = make_desc(dom, device, stream, self._alloc)
        h = C.c_void_p()
        _check(L.rwmi_create_domain(C.byref(self._desc), C.byref(h)))
        self.h = h
        self.nparticles = 0
        self.nw = 0

    def close(self):
        if getattr(self, "h", None):
            # the library takes a domain out of its batch before freeing it
            bt = getattr(self, "_batch", None)
            if bt is not None and self in bt.members:
                bt.members.remove(self)
            self._batch = None
            self.L.rwmi_destroy_domain(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, st):
        _check(st, self.h)

    def add_particle(self, p):
        b = np.ascontiguousarray(np.asarray(p["b"], float).ravel())
        k = np.ascontiguousarray(np.asarray(p["k"], float).ravel())
        m = MetaballDesc()
        m.n_ctrl = k.size
        m.offsets = _dptr(b)
        m.weights = _dptr(k)
        c = p["centre"]
        amp = p.get("amp", (0, 0, 0))
        vel = p.get("vel", (0, 0, 0))
        for a in range(3):
            m.centre[a] = float(c[a])
            m.amplitude[a] = float(amp[a])
            m.velocity[a] = float(vel[a])
        m.motion = MOTION[p.get("motion", "static")]
        m.period = float(p.get("period", 1.0))
        m.phase = float(p.get("phase", 0.0))
        out = C.c_int32()
        self._ck(self.L.rwmi_add_metaball_particle(self.h, C.byref(m), C.byref(out)))
        self.nparticles += 1
        return out.value

    def set_coupling(self, dem):
        """Two-way coupling of the particles added with motion "coupled"
        (Eq. 4-11); after adding the particles, before seeding."""
        c = coupling_desc(dem)
        self._ck(self.L.rwmi_set_coupling(self.h, C.byref(c)))

    def set_fluid_coupling(self, scheme):
        """"psm" (partially saturated cells) or "ibb" (interpolated
        bounce-back, Eq. 23-27); before the first step."""
        self._ck(self.L.rwmi_set_fluid_coupling(self.h, {"psm": 0, "ibb": 1}[scheme]))

    def particle_state(self, p):
        o = np.zeros(32)
        self._ck(self.L.rwmi_read_particle_state(self.h, int(p), o.ctypes.data_as(C.c_void_p)))
        return {"c": o[0:3].copy(), "v": o[3:6].copy(), "q": o[6:10].copy(), "L": o[10:13].copy(),
                "w": o[13:16].copy(), "Fh": o[16:19].copy(), "Th": o[19:22].copy(), "mass": float(o[22]),
                "I": o[23:32].reshape(3, 3).copy()}

    def set_particle_motion(self, p, v, L):
        v = np.ascontiguousarray(np.asarray(v, float).ravel())
        L = np.ascontiguousarray(np.asarray(L, float).ravel())
        assert v.size == 3 and L.size == 3
        self._ck(self.L.rwmi_set_particle_motion(self.h, int(p), v.ctypes.data_as(C.c_void_p),
                                                 L.ctypes.data_as(C.c_void_p)))

    def seed(self, s, n, check=True):
        sd = SeedDesc()
        sd.kind = SEED_KIND[s["kind"]]
        c = s.get("centre", (0, 0, 0))
        ref = s.get("ref", [0.5 * v for v in self.n])
        for a in range(3):
            sd.centre[a] = float(c[a])
            sd.ref[a] = float(ref[a])
        sd.sigma = float(s.get("sigma", 1.0))
        band = s.get("band", (2, 0.0, 1.0))
        sd.band_axis, sd.band_lo, sd.band_hi = int(band[0]), float(band[1]), float(band[2])
        xyz = None
        if sd.kind == 3:
            xyz = np.ascontiguousarray(np.asarray(s["xyz"], float).reshape(-1))
            sd.xyz = _dptr(xyz)
        sd.max_attempts = int(s.get("max_attempts", 64))
        sd.remove_inside = int(s.get("remove_inside", 0))
        out = C.c_uint64()
        st = self.L.rwmi_seed_walkers(self.h, C.byref(sd), int(n), C.byref(out))
        self.nw = int(out.value)
        if check:
            self._ck(st)
        return self.nw

    def step(self, n=1):
        self._ck(self.L.rwmi_step(self.h, int(n)))

    def sync(self):
        self._ck(self.L.rwmi_synchronize(self.h))

    def set(self, key, value):
        self._ck(self.L.rwmi_debug_set(self.h, KEY[key], int(value)))

    def sizes(self):
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        self._ck(self.L.rwmi_query_sizes(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def moments(self, noalloc=False):
        """FP64 moments; noalloc=True reads them through the allocation-free
        entry point (same kernels, scratch in the library's device array)."""
        m = Moments()
        f = self.L.rwmi_read_moments_noalloc if noalloc else self.L.rwmi_read_moments
        self._ck(f(self.h, C.byref(m)))
        return dict(step=int(m.step), n_walkers=int(m.n_walkers), sum=np.array(m.sum[:]), sumsq=np.array(m.sumsq[:]),
                    mass=m.mass, momentum=np.array(m.momentum[:]), fluid_u=np.array(m.fluid_u[:]),
                    particle_v=np.array(m.particle_v[:]), solid_volume=m.solid_volume,
                    counters=dict(type2=int(m.type2), type4=int(m.type4), bisect_fail=int(m.bisect_fail),
                                  refill_fallback=int(m.refill_fallback),
                                  returned_to_origin=int(m.returned_to_origin), wall_reflect=int(m.wall_reflect)),
                    near_surface=int(m.near_surface), contact_misses=int(m.contact_misses))

    def occupancy(self):
        ns = np.empty(self.N, np.uint32)
        self._ck(self.L.rwmi_read_occupancy(self.h, ns.ctypes.data_as(C.c_void_p)))
        return ns.reshape(self.n[::-1])

    def profile(self, axis=2):
        """Walkers per layer along `axis` (exact counts, n[axis] entries)."""
        c = np.empty(self.n[axis], np.uint64)
        self._ck(self.L.rwmi_read_profile(self.h, int(axis), c.ctypes.data_as(C.c_void_p)))
        return c

    def velocity(self):
        u = np.empty(3 * self.N)
        rho = np.empty(self.N)
        self._ck(self.L.rwmi_read_velocity(self.h, u.ctypes.data_as(C.c_void_p), rho.ctypes.data_as(C.c_void_p)))
        sh = self.n[::-1]
        return u.reshape(3, *sh), rho.reshape(sh)

    def walkers(self):
        _, m, _ = self.sizes()
        cell = np.empty(max(m, 1), np.int32)
        off = np.empty(max(3 * m, 1))
        img = np.empty(max(3 * m, 1), np.int32)
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self._ck(self.L.rwmi_read_walkers(self.h, vp(cell), vp(off), vp(img)))
        return cell[:m].copy(), off[:3 * m].reshape(3, m).copy(), img[:3 * m].reshape(3, m).copy()

    def distributions(self):
        f = np.empty(19 * self.N)
        self._ck(self.L.rwmi_read_distributions(self.h, f.ctypes.data_as(C.c_void_p)))
        return f.reshape(19, *self.n[::-1])

    def kernel_times(self):
        """(total ms, launches, of which with a fluid update, of which with a
        walker step) of the step launches timed since the last call."""
        ms, n, nf, nw = C.c_double(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        self._ck(self.L.rwmi_read_kernel_times(self.h, C.byref(ms), C.byref(n), C.byref(nf), C.byref(nw)))
        return ms.value, int(n.value), int(nf.value), int(nw.value)

    def coupling_times(self):
        """(ms, count) of the particle updates and of the prologues timed
        since the last call (coupled particles with timing on)."""
        mu, nu, mp, npr = C.c_double(), C.c_uint64(), C.c_double(), C.c_uint64()
        self._ck(self.L.rwmi_read_coupling_times(self.h, C.byref(mu), C.byref(nu), C.byref(mp), C.byref(npr)))
        return (mu.value, int(nu.value)), (mp.value, int(npr.value))


def build_domain(cfg, device=0, use_torch=True, seed_walkers=True):
    """Domain with the particles (and walkers) of a generated configuration."""
    d = Domain(cfg["domain"], device=device, use_torch=use_torch)
    for p in cfg.get("particles", []):
        d.add_particle(p)
    if cfg["domain"].get("coupling") == "ibb":
        d.set_fluid_coupling("ibb")
    if cfg.get("dem"):
        d.set_coupling(cfg["dem"])
    if seed_walkers and cfg.get("walkers") and cfg["walkers"].get("n", 0) > 0:
        d.seed(cfg["walkers"], cfg["walkers"]["n"])
    return d


class Batch:
    """Many domains stepped together (one launch per kernel per step)."""

    def __init__(self, device=0, use_torch=True):
        L = lib()
        self.L = L
        torch = _torch_gpu() if use_torch else None
        self._torch_stream = torch.cuda.Stream(device=device) if torch is not None else None
        stream = C.c_void_p(self._torch_stream.cuda_stream) if self._torch_stream is not None else None
        h = C.c_void_p()
        _check(L.rwmi_batch_create(int(device), stream, C.byref(h)))
        self.h = h
        self.members = []

    def _ck(self, st):
        _check(st, None)

    def add(self, dom):
        self._ck(self.L.rwmi_batch_add(self.h, dom.h))
        self.members.append(dom)
        dom._batch = self

    def remove(self, dom):
        self._ck(self.L.rwmi_batch_remove(self.h, dom.h))
        self.members.remove(dom)
        dom._batch = None

    def step(self, n=1):
        self._ck(self.L.rwmi_batch_step(self.h, int(n)))

    def set(self, key, value):
        self._ck(self.L.rwmi_batch_set(self.h, KEY[key], int(value)))

    def sync(self):
        self._ck(self.L.rwmi_batch_synchronize(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.rwmi_batch_destroy(self.h)
            self.h = None
            for d in self.members:
                d._batch = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dispersion_fit(t, sigma2, two_r, u_slip, phi, i0=0):
    """K, D_alpha and offset of Eq. 38-40 from a moment series (library host code)."""
    t = np.ascontiguousarray(t, float)
    s2 = np.ascontiguousarray(sigma2, float)
    K, Da, off = C.c_double(), C.c_double(), C.c_double()
    _check(lib().rwmi_dispersion_fit(t.ctypes.data_as(C.c_void_p), s2.ctypes.data_as(C.c_void_p), t.size, int(i0),
                                     float(two_r), float(u_slip), float(phi), C.byref(K), C.byref(Da), C.byref(off)))
    return K.value, Da.value, off.value


def moments_struct(m):
    """A Moments structure holding the fields of a moments dict."""
    r = Moments()
    r.step = int(m["step"])
    r.n_walkers = int(m["n_walkers"])
    for a in range(3):
        r.sum[a] = float(m["sum"][a])
        r.sumsq[a] = float(m["sumsq"][a])
        r.momentum[a] = float(m["momentum"][a])
        r.fluid_u[a] = float(m["fluid_u"][a])
        r.particle_v[a] = float(m["particle_v"][a])
    r.mass = float(m["mass"])
    r.solid_volume = float(m["solid_volume"])
    return r


def dispersion_from_moments(series, n_nodes, two_r, disp_axis=2, flow_axis=0, i0=None):
    """Eq. 38-40 from a list of moments dicts through the library: (sigma2
    series, dict of u_slip, phi, K, D_alpha, offset)."""
    n = len(series)
    arr = (Moments * max(n, 1))()
    for i, m in enumerate(series):
        arr[i] = moments_struct(m)
    i0 = n // 2 if i0 is None else int(i0)
    s2 = np.empty(max(n, 1))
    out = Dispersion()
    _check(lib().rwmi_dispersion_from_moments(arr, n, i0, int(disp_axis), int(flow_axis), int(n_nodes), float(two_r),
                                              s2.ctypes.data_as(C.c_void_p), C.byref(out)))
    return s2[:n], dict(u_slip=out.u_slip, phi=out.phi, K=out.K, D_alpha=out.D_alpha, offset=out.offset)


def gaussian_fit(x, y):
    """(amp, mean, var) of the least-squares Gaussian through (x, y) (library host code)."""
    x = np.ascontiguousarray(x, float)
    y = np.ascontiguousarray(y, float)
    a, m, v = C.c_double(), C.c_double(), C.c_double()
    _check(lib().rwmi_gaussian_fit(x.ctypes.data_as(C.c_void_p), y.ctypes.data_as(C.c_void_p), x.size, C.byref(a),
                                   C.byref(m), C.byref(v)))
    return a.value, m.value, v.value


def device_normals(seed, t, purpose, n, device=0):
    z = np.empty(3 * n)
    _check(lib().rwmi_device_normals(int(device), int(seed), int(t), int(purpose), int(n),
                                     z.ctypes.data_as(C.c_void_p)))
    return z.reshape(n, 3)


def stream_probe(streams, tiled, src, dst, stream=None):
    """One launch of the bandwidth probe on device tensors src and dst of
    streams * n floats or halves each (n = src.numel() // streams), on
    `stream` (a torch stream; default the current one)."""
    import torch
    n = src.numel() // int(streams)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().rwmi_stream_probe(int(streams), int(src.element_size()), int(bool(tiled)), n,
                                   C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                   C.c_void_p(s.cuda_stream)))
