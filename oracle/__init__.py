"""ctypes wrapper around the FP64 CPU oracle (``rwmi_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library and its Python
binding never do.  It shares no code with the HIP path: inputs come from the
seeded generators (which hold none of the method's arithmetic) and are handed
to both sides as plain arrays.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rwmi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-Wall", "-Wno-unused-function"]


def build(force=False):
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [ip, ip, dp, dp, C.c_double, dp, C.c_double, C.c_double, dp, C.c_uint64]
        L.orc_destroy.argtypes = [P]
        L.orc_set_max_bisect.argtypes = [P, C.c_int]
        L.orc_add_particle.restype = C.c_int
        L.orc_add_particle.argtypes = [P, C.c_int, dp, dp, dp, C.c_int, dp, C.c_double, C.c_double, dp]
        L.orc_step.argtypes = [P, C.c_int]
        L.orc_seed.restype = C.c_int64
        L.orc_seed.argtypes = [P, C.c_int, dp, C.c_double, C.c_int, C.c_double, C.c_double, C.c_void_p,
                               C.c_int64, C.c_int, C.c_int, dp]
        L.orc_occupancy.argtypes = [P, up]
        L.orc_moments.argtypes = [P, dp]
        for name in ("orc_num_nodes", "orc_num_walkers", "orc_time"):
            getattr(L, name).restype = C.c_int64
            getattr(L, name).argtypes = [P]
        L.orc_counters.argtypes = [P, u64p]
        L.orc_get_ref.argtypes = [P, dp]
        L.orc_get_f.argtypes = [P, dp]
        L.orc_set_f.argtypes = [P, dp]
        L.orc_get_fields.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_walkers.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_walkers.argtypes = [P, C.c_int64, ip, dp, dp]
        L.orc_philox.argtypes = [up, up, up]
        L.orc_ln_export.restype = C.c_double
        L.orc_ln_export.argtypes = [C.c_double]
        L.orc_sincos2pi.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_normals.argtypes = [up, up, dp]
        L.orc_normals_batch.argtypes = [C.c_uint32, C.c_uint32, up, C.c_int64, dp]
        L.orc_feq.argtypes = [C.c_double, dp, dp]
        L.orc_lattice.argtypes = [ip, dp]
        L.orc_collide_node.argtypes = [P, dp, C.c_double, dp, dp, C.POINTER(C.c_double), dp]
        L.orc_particle_M.restype = C.c_double
        L.orc_particle_M.argtypes = [P, C.c_int, C.c_int64, ip, dp]
        L.orc_particle_grad.argtypes = [P, C.c_int, C.c_int64, ip, dp, dp]
        L.orc_particle_pose.argtypes = [P, C.c_int, C.c_int64, dp, dp]
        L.orc_particle_rb.restype = C.c_double
        L.orc_particle_rb.argtypes = [P, C.c_int]
        L.orc_bisect_segment.restype = C.c_double
        L.orc_bisect_segment.argtypes = [P, C.c_int, C.c_int64, ip, dp, dp, C.c_double, C.c_double,
                                         C.c_int, C.POINTER(C.c_int)]
        L.orc_reflect.argtypes = [dp, dp, dp]
        L.orc_dispersion_from_moments.restype = C.c_int
        L.orc_dispersion_from_moments.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                                  C.c_void_p, dp]
        L.orc_profile.argtypes = [P, C.c_int, u64p]
        L.orc_gaussian_fit.restype = C.c_int
        L.orc_gaussian_fit.argtypes = [dp, dp, C.c_int, dp]
        L.orc_set_dem.restype = C.c_int
        L.orc_set_dem.argtypes = [P, dp]
        L.orc_dem_state.argtypes = [P, C.c_int, dp]
        L.orc_dem_set_motion.argtypes = [P, C.c_int, dp, dp]
        L.orc_set_ibb.restype = C.c_int
        L.orc_set_ibb.argtypes = [P, C.c_int]
        L.orc_ibb_ud.argtypes = [C.c_double, dp, dp, dp, dp]
        L.orc_ibb_q.restype = C.c_double
        L.orc_ibb_q.argtypes = [P, C.c_int, C.c_int64, ip, C.c_int, dp]
        L.orc_get_smap.argtypes = [P, ip]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_dispersion_fit.restype = C.c_int
        L.orc_dispersion_fit.argtypes = [dp, dp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _d(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def _raise(msg):
    raise ValueError(msg)


DEM_KEYS = ("rho_p", "g", "drive_amp", "drive_period", "drive_dir", "kn", "kt", "eta_n", "eta_t", "mu", "Rs",
            "nsub", "coupling")
DEM_DEFAULTS = {"g": (0.0, 0.0, 0.0), "drive_amp": 0.0, "drive_period": 5000.0, "drive_dir": (1.0, 0.0, 0.0),
                "kt": 0.0, "eta_n": 0.0, "eta_t": 0.0, "mu": 0.0, "nsub": 100, "coupling": 1}


def dem_params(dem):
    """The 17 doubles of the coupling parameters, in the C layout."""
    v = dict(DEM_DEFAULTS, **dem)
    out = []
    for k in DEM_KEYS:
        x = v[k]
        out.extend(np.ravel(x).astype(float).tolist())
    assert len(out) == 17
    return _d(out, 17)


BC_PERIODIC, BC_WALL = 0, 1
MOTION = {"static": 0, "sinusoid": 1, "const_vel": 2, "coupled": 3}
SEED_KIND = {"uniform": 0, "gaussian": 1, "band": 2, "explicit": 3}
COUNTERS = ("type2", "type4", "bisect_fail", "refill_fallback", "returned_to_origin", "wall_reflect")


class Oracle:
    """One simulation domain of the oracle; mirrors the C-ABI's operations.

    ``dom`` is the plain dictionary produced by the workload generators:
    n, bc, wall_lo, wall_hi, tau, F, D, rho0, u0, seed."""

    def __init__(self, dom):
        self.L = lib()
        n = np.asarray(dom["n"], dtype=np.int32)
        bc = np.asarray([BC_WALL if b in ("wall", 1) else BC_PERIODIC for b in dom.get("bc", ["periodic"] * 3)],
                        dtype=np.int32)
        self.n = tuple(int(v) for v in n)
        self.bc = tuple("wall" if b == BC_WALL else "periodic" for b in bc)
        self.N = int(np.prod(self.n))
        self.h = self.L.orc_create(n, bc, _d(dom.get("wall_lo", np.zeros(9)), 9), _d(dom.get("wall_hi", np.zeros(9)), 9),
                                   float(dom["tau"]), _d(dom.get("F", (0, 0, 0)), 3), float(dom.get("D", 0.0)),
                                   float(dom.get("rho0", 1.0)), _d(dom.get("u0", (0, 0, 0)), 3),
                                   int(dom.get("seed", 0)) & (2**64 - 1))
        self.nparticles = 0

    def __del__(self):
        try:
            if self.h:
                self.L.orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_max_bisect(self, m):
        self.L.orc_set_max_bisect(self.h, int(m))

    def add_particle(self, p):
        b = _d(p["b"])
        k = _d(p["k"])
        r = self.L.orc_add_particle(self.h, k.size, b, k, _d(p["centre"], 3), MOTION[p.get("motion", "static")],
                                    _d(p.get("amp", (0, 0, 0)), 3), float(p.get("period", 1.0)),
                                    float(p.get("phase", 0.0)), _d(p.get("vel", (0, 0, 0)), 3))
        if r < 0:
            raise ValueError("oracle: too many particles or empty particle")
        self.nparticles += 1
        return r

    def set_dem(self, dem):
        """Two-way coupling of the particles added with motion "coupled"
        (Eq. 4-11); call after adding the particles, before seeding."""
        self.L.orc_set_dem(self.h, dem_params(dem)) == 0 or _raise("oracle: bad coupling parameters")

    def set_ibb(self, on=True):
        """Interpolated bounce-back coupling (Eq. 23-27) instead of the
        partially saturated cells; before the first step."""
        self.L.orc_set_ibb(self.h, int(bool(on))) == 0 or _raise("oracle: the coupling is chosen before stepping")

    def ibb_q(self, p, t, cell, o):
        dlw = np.zeros(3)
        q = self.L.orc_ibb_q(self.h, int(p), int(t), np.asarray(cell, np.int32), int(o), dlw)
        return q, dlw

    def smap(self):
        out = np.empty(self.N, np.int32)
        self.L.orc_get_smap(self.h, out)
        return out.reshape(self.n[::-1])

    def dem_state(self, p):
        o = np.zeros(32)
        self.L.orc_dem_state(self.h, int(p), o)
        return {"c": o[0:3].copy(), "v": o[3:6].copy(), "q": o[6:10].copy(), "L": o[10:13].copy(),
                "w": o[13:16].copy(), "Fh": o[16:19].copy(), "Th": o[19:22].copy(), "mass": float(o[22]),
                "I": o[23:32].reshape(3, 3).copy()}

    def dem_set_motion(self, p, v, L):
        self.L.orc_dem_set_motion(self.h, int(p), _d(v, 3), _d(L, 3))

    def seed(self, s, n):
        kind = SEED_KIND[s["kind"]]
        xyz = None
        ptr = None
        if kind == 3:
            xyz = _d(s["xyz"], 3 * n)
            ptr = xyz.ctypes.data_as(C.c_void_p)
        ref = _d(s.get("ref", [0.5 * v for v in self.n]), 3)
        band = s.get("band", (2, 0.0, 1.0))
        m = self.L.orc_seed(self.h, kind, _d(s.get("centre", (0, 0, 0)), 3), float(s.get("sigma", 1.0)),
                            int(band[0]), float(band[1]), float(band[2]), ptr, int(n),
                            int(s.get("max_attempts", 64)), int(s.get("remove_inside", 0)), ref)
        return int(m)

    def step(self, n=1):
        self.L.orc_step(self.h, int(n))

    @property
    def t(self):
        return int(self.L.orc_time(self.h))

    @property
    def nw(self):
        return int(self.L.orc_num_walkers(self.h))

    def f(self):
        out = np.empty(19 * self.N)
        self.L.orc_get_f(self.h, out)
        return out.reshape(19, *self.n[::-1])

    def set_f(self, f):
        self.L.orc_set_f(self.h, _d(f, 19 * self.N))

    def fields(self):
        rho = np.empty(self.N)
        u = np.empty(3 * self.N)
        eps = np.empty(self.N)
        us = np.empty(3 * self.N)
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self.L.orc_get_fields(self.h, vp(rho), vp(u), vp(eps), vp(us))
        sh = self.n[::-1]
        return dict(rho=rho.reshape(sh), u=u.reshape(3, *sh), eps=eps.reshape(sh), us=us.reshape(3, *sh))

    def walkers(self):
        m = self.nw
        cell = np.empty(max(m, 1), np.int32)
        off = np.empty(max(3 * m, 1))
        img = np.empty(max(3 * m, 1), np.int32)
        vp = lambda a: a.ctypes.data_as(C.c_void_p)
        self.L.orc_get_walkers(self.h, vp(cell), vp(off), vp(img))
        return cell[:m].copy(), off[:3 * m].reshape(3, m).copy(), img[:3 * m].reshape(3, m).copy()

    def set_walkers(self, cell, off, ref):
        cell = np.ascontiguousarray(cell, np.int32)
        self.L.orc_set_walkers(self.h, cell.size, cell, _d(off, 3 * cell.size), _d(ref, 3))

    def occupancy(self):
        ns = np.empty(self.N, np.uint32)
        self.L.orc_occupancy(self.h, ns)
        return ns.reshape(self.n[::-1])

    def moments(self):
        out = np.empty(19)
        self.L.orc_moments(self.h, out)
        return dict(n_walkers=out[0], sum=out[1:4].copy(), sumsq=out[4:7].copy(), mass=out[7],
                    momentum=out[8:11].copy(), fluid_u=out[11:14].copy(), particle_v=out[14:17].copy(),
                    solid_volume=out[17], step=out[18])

    def ref(self):
        """Reference point of the walker moments (set at seeding)."""
        r = np.empty(3)
        self.L.orc_get_ref(self.h, r)
        return r

    def profile(self, axis=2):
        """Walkers per layer along `axis`."""
        c = np.empty(self.n[axis], np.uint64)
        self.L.orc_profile(self.h, int(axis), c)
        return c

    def counters(self):
        c = np.zeros(8, np.uint64)
        self.L.orc_counters(self.h, c)
        return {k: int(c[i]) for i, k in enumerate(COUNTERS)}

    # single-particle helpers for the pins
    def particle_M(self, p, t, cell, x):
        return self.L.orc_particle_M(self.h, int(p), int(t), np.asarray(cell, np.int32), _d(x, 3))

    def particle_grad(self, p, t, cell, x):
        g = np.empty(3)
        self.L.orc_particle_grad(self.h, int(p), int(t), np.asarray(cell, np.int32), _d(x, 3), g)
        return g

    def particle_pose(self, p, t):
        c = np.empty(3)
        v = np.empty(3)
        self.L.orc_particle_pose(self.h, int(p), int(t), c, v)
        return c, v

    def particle_rb(self, p):
        return self.L.orc_particle_rb(self.h, int(p))

    def bisect(self, p, t, cell, a0, direction, s_out, s_in, imax=200):
        ok = C.c_int(0)
        s = self.L.orc_bisect_segment(self.h, int(p), int(t), np.asarray(cell, np.int32), _d(a0, 3),
                                      _d(direction, 3), float(s_out), float(s_in), int(imax), C.byref(ok))
        return bool(ok.value), s

    def collide_node(self, f, eps, us):
        out = np.empty(19)
        u = np.empty(3)
        rho = C.c_double(0)
        self.L.orc_collide_node(self.h, _d(f, 19), float(eps), _d(us, 3), out, C.byref(rho), u)
        return out, rho.value, u


def philox(ctr, key):
    out = np.empty(4, np.uint32)
    lib().orc_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def ln(u):
    return lib().orc_ln_export(float(u))


def sincos2pi(u):
    s = C.c_double()
    c = C.c_double()
    lib().orc_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def normals(t, purpose, seed, n):
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32)
    z = np.empty(3 * n)
    lib().orc_normals_batch(int(t), int(purpose), key, int(n), z)
    return z.reshape(n, 3)


def feq(rho, u):
    out = np.empty(19)
    lib().orc_feq(float(rho), _d(u, 3), out)
    return out


def lattice():
    e = np.empty(57, np.int32)
    w = np.empty(19)
    lib().orc_lattice(e, w)
    return e.reshape(19, 3), w


def reflect(ti, g):
    tr = np.empty(3)
    lib().orc_reflect(_d(ti, 3), _d(g, 3), tr)
    return tr


def dispersion_fit(t, sigma2, two_r, u_slip, phi, i0=0):
    K = C.c_double()
    Da = C.c_double()
    t = _d(t)
    s2 = _d(sigma2)
    r = lib().orc_dispersion_fit(t, s2, t.size, int(i0), float(two_r), float(u_slip), float(phi), C.byref(K),
                                 C.byref(Da))
    if r != 0:
        raise ValueError("oracle dispersion fit: invalid input")
    return K.value, Da.value


MOMENT_FIELDS = ("n_walkers", "sum", "sumsq", "mass", "momentum", "fluid_u", "particle_v", "solid_volume", "step")


def ibb_ud(q, uf, uff, uw):
    ud = np.zeros(3)
    lib().orc_ibb_ud(float(q), _d(uf, 3), _d(uff, 3), _d(uw, 3), ud)
    return ud


def moments_record(m):
    """The 19-double moment record (orc_moments layout) of a moments dict."""
    r = np.zeros(19)
    r[0] = m["n_walkers"]
    r[1:4] = m["sum"]
    r[4:7] = m["sumsq"]
    r[7] = m["mass"]
    r[8:11] = m["momentum"]
    r[11:14] = m["fluid_u"]
    r[14:17] = m["particle_v"]
    r[17] = m["solid_volume"]
    r[18] = m["step"]
    return r


def dispersion_from_moments(series, n_nodes, two_r, disp_axis=2, flow_axis=0, i0=None):
    """Eq. 38-40 from a list of moments dicts: (sigma2 series, dict of
    u_slip, phi, K, D_alpha, offset)."""
    rec = np.ascontiguousarray(np.stack([moments_record(m) for m in series]).ravel())
    n = len(series)
    i0 = n // 2 if i0 is None else int(i0)
    s2 = np.empty(n)
    out = np.empty(5)
    r = lib().orc_dispersion_from_moments(rec, n, i0, int(disp_axis), int(flow_axis), float(n_nodes), float(two_r),
                                          s2.ctypes.data_as(C.c_void_p), out)
    if r != 0:
        raise ValueError("oracle dispersion: invalid input")
    return s2, dict(u_slip=out[0], phi=out[1], K=out[2], D_alpha=out[3], offset=out[4])


def gaussian_fit(x, y):
    """(A, mu, s2) of the least-squares Gaussian through (x, y)."""
    out = np.empty(3)
    x = _d(x)
    y = _d(y)
    if lib().orc_gaussian_fit(x, y, x.size, out) != 0:
        raise ValueError("oracle gaussian fit: invalid input")
    return out[0], out[1], out[2]


def set_threads(n):
    """Threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def build_domain(cfg):
    """Oracle domain with the particles of a generated configuration."""
    o = Oracle(cfg["domain"])
    for p in cfg.get("particles", []):
        o.add_particle(p)
    if cfg.get("dem"):
        o.set_dem(cfg["dem"])
    if cfg["domain"].get("coupling") == "ibb":
        o.set_ibb(True)
    return o
