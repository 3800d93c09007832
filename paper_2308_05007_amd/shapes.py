"""Particle shape features of Sec. 4 (Eq. 41-44) and the Spearman rank
correlation of Eq. 45, for bodies given by an implicit function.

A body is a level set g(x) <= 0 of a field g whose zero set is the surface.
For a metaball (Eq. 3) g = M^(-1/2) - 1, which is r/sqrt(k) - 1 for one
control point: zero on the surface M = 1 and smooth across it.  The first-
order distance to the surface is d = g / |grad g| (negative inside).

Integrals over the body are taken on a grid of spacing h with smoothed
indicators of d, which makes them second-order accurate in h:
  volume        sum of clamp(1/2 - d/h, 0, 1) h^3 (the cell's inside fraction
                for a plane surface),
  surface area  sum of delta_e(d) h^3 with delta_e(d) = (1 + cos(pi d/e)) / (2e)
                for |d| < e = 1.5 h (the coarea formula),
and the same in two dimensions for a projection (area and perimeter of the
shadow, whose field is the minimum of g along the projection rays).

Features (Sec. 4):
  sphericity   phi  = A_ve / A, A_ve the area of the volume-equivalent sphere (Eq. 41)
  circularity  C_c  = pi D_s / P_p, P_p the perimeter of the projection of
                      largest area (Eq. 42)
  D_ns         D_n / D_s, D_n = (6 V / pi)^(1/3), D_s = sqrt(4 A_m / pi) (Eq. 43)
  CSF          L_s / sqrt(L_i L_l), the extents along the principal axes of
               inertia, shortest / intermediate / longest (Eq. 44)
  A_m          the largest projected area over directions (a Fibonacci set
               refined around its best direction)
"""
import math

import numpy as np


# ------------------------------------------------------------------ bodies
class Metaball:
    """The body M(x) >= 1 of control points b (n x 3) with weights k (Eq. 3)."""

    def __init__(self, b, k):
        self.b = np.asarray(b, float).reshape(-1, 3)
        self.k = np.asarray(k, float).ravel()
        r = np.sqrt((self.b ** 2).sum(1)).max()
        self.radius = r + math.sqrt(self.k.sum())  # bounding radius: M <= 1 beyond it

    def M(self, x):
        M = np.zeros(x.shape[:-1])
        for bi, ki in zip(self.b, self.k):
            r2 = ((x - bi) ** 2).sum(-1)
            with np.errstate(divide="ignore"):
                M = M + ki / r2
        return M

    def g(self, x):
        M = self.M(x)
        with np.errstate(divide="ignore"):
            return np.where(np.isinf(M), -1.0, M ** -0.5 - 1.0)

    def scaled(self, s):
        """The same shape scaled by s (offsets x s, weights x s^2: M(x/s) exactly)."""
        return Metaball(self.b * s, self.k * s * s)

    def rotated(self, R):
        return Metaball(self.b @ np.asarray(R).T, self.k)


class Ellipsoid:
    """x^2/a^2 + y^2/b^2 + z^2/c^2 <= 1 (closed-form checks of the features)."""

    def __init__(self, a, b, c, R=None):
        self.ax = np.array([a, b, c], float)
        self.R = np.eye(3) if R is None else np.asarray(R, float)
        self.radius = float(self.ax.max())

    def g(self, x):
        y = x @ self.R  # body coordinates
        return np.sqrt(((y / self.ax) ** 2).sum(-1)) - 1.0

    def rotated(self, R):
        return Ellipsoid(*self.ax, R=np.asarray(R) @ self.R)


# ------------------------------------------------------------------ grids
def _grad(f, x, eps=1e-5):
    g = np.empty(x.shape)
    for a in range(x.shape[-1]):
        e = np.zeros(x.shape[-1])
        e[a] = eps
        g[..., a] = (f(x + e) - f(x - e)) / (2 * eps)
    return g


def _grid(radius, h, dim=3):
    m = int(math.ceil((radius + 3 * h) / h))
    ax = (np.arange(-m, m + 1) * h)
    return np.stack(np.meshgrid(*(ax,) * dim, indexing="ij"), -1)


def _dist(f, x):
    """First-order signed distance g / |grad g| (negative inside)."""
    gv = f(x)
    gn = np.sqrt((_grad(f, x) ** 2).sum(-1))
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.where(gn > 0, gv / gn, np.where(gv <= 0, -np.inf, np.inf))
    return d


def _heaviside(d, h):
    return np.clip(0.5 - d / h, 0.0, 1.0)


def _delta(d, h):
    e = 1.5 * h
    out = np.zeros_like(d)
    m = np.abs(d) < e
    out[m] = (1.0 + np.cos(np.pi * d[m] / e)) / (2 * e)
    return out


def volume_area(body, h=0.1, chunk=200000):
    """Volume and surface area of the body."""
    X = _grid(body.radius, h).reshape(-1, 3)
    V = A = 0.0
    for i in range(0, len(X), chunk):
        d = _dist(body.g, X[i:i + chunk])
        V += _heaviside(d, h).sum() * h ** 3
        A += _delta(d, h).sum() * h ** 3
    return V, A


def _frame(n):
    """Orthonormal (e1, e2, n) with n the given direction."""
    n = np.asarray(n, float) / np.linalg.norm(n)
    t = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, t)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(n, e1), n


def projection(body, n, h=0.1):
    """Area and perimeter of the body's projection along direction n: the
    shadow's field is the minimum of g over each projection ray."""
    e1, e2, nn = _frame(n)
    r = body.radius + 3 * h
    m = int(math.ceil(r / h))
    t = np.arange(-m, m + 1) * h

    def s(p2):  # p2: (..., 2) plane coordinates -> minimum of g along the ray
        P = p2[..., 0, None, None] * e1 + p2[..., 1, None, None] * e2 + t[:, None] * nn
        return body.g(P).min(-1)

    U = _grid(body.radius, h, dim=2).reshape(-1, 2)
    out_a = out_p = 0.0
    for i in range(0, len(U), 4000):
        d = _dist(s, U[i:i + 4000])
        out_a += _heaviside(d, h).sum() * h * h
        out_p += _delta(d, h).sum() * h * h
    return out_a, out_p


def fibonacci_directions(n):
    """n unit vectors spread over the upper half sphere (a projection and its
    opposite are the same)."""
    i = np.arange(n) + 0.5
    z = i / n
    phi = np.pi * (1 + 5 ** 0.5) * i
    rr = np.sqrt(1 - z * z)
    return np.stack([rr * np.cos(phi), rr * np.sin(phi), z], -1)


def max_projection(body, h=0.1, n_dirs=48, refine=2):
    """The largest projected area and its direction: the best of a
    Fibonacci set, then refined on rings around it."""
    best_a, best_n = -1.0, None
    for n in fibonacci_directions(n_dirs):
        a, _ = projection(body, n, h)
        if a > best_a:
            best_a, best_n = a, n
    step = math.acos(1 - 1.0 / n_dirs) * 1.5
    for _ in range(refine):
        e1, e2, nn = _frame(best_n)
        for k in range(8):
            ang = 2 * np.pi * k / 8
            n = math.cos(step) * nn + math.sin(step) * (math.cos(ang) * e1 + math.sin(ang) * e2)
            a, _ = projection(body, n, h)
            if a > best_a:
                best_a, best_n = a, n
        step *= 0.5
    return best_a, best_n


def principal_extents(body, h=0.1):
    """Extents of the body along its principal axes of inertia, sorted
    shortest first, from the surface points x - d grad g / |grad g| of the
    cells next to the surface."""
    X = _grid(body.radius, h).reshape(-1, 3)
    d = _dist(body.g, X)
    w = _heaviside(d, h)
    c = (X * w[:, None]).sum(0) / w.sum()
    Y = X - c
    I = (Y[:, :, None] * Y[:, None, :] * w[:, None, None]).sum(0)
    _, vecs = np.linalg.eigh(I)
    near = np.abs(d) < h
    gr = _grad(body.g, X[near])
    P = X[near] - d[near, None] * gr / np.linalg.norm(gr, axis=1)[:, None] - c
    ext = [(P @ v).max() - (P @ v).min() for v in vecs.T]
    return sorted(ext)


def features(body, h=0.1, n_dirs=48):
    """Shape features of Sec. 4 (Eq. 41-44) and the quantities they come from."""
    V, A = volume_area(body, h)
    Am, nbest = max_projection(body, h, n_dirs)
    _, Pp = projection(body, nbest, h)
    Dn = (6.0 * V / math.pi) ** (1.0 / 3.0)
    Ds = math.sqrt(4.0 * Am / math.pi)
    Ls, Li, Ll = principal_extents(body, h)
    Ave = math.pi * Dn * Dn
    return {"volume": V, "area": A, "A_m": Am, "P_p": Pp, "D_n": Dn, "D_s": Ds, "axes": (Ls, Li, Ll),
            "sphericity": Ave / A, "C_c": math.pi * Ds / Pp, "D_ns": Dn / Ds, "CSF": Ls / math.sqrt(Li * Ll)}


# ------------------------------------------------------------------ Eq. 45
def ranks(x):
    """Ranks 1..n, ties sharing the mean of their positions."""
    x = np.asarray(x, float)
    order = np.argsort(x, kind="mergesort")
    r = np.empty(x.size)
    i = 0
    while i < x.size:
        j = i
        while j + 1 < x.size and x[order[j + 1]] == x[order[i]]:
            j += 1
        r[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return r


def spearman(x, y):
    """Spearman's rank correlation: the Pearson correlation of the ranks.
    Without ties this is Eq. 45, 1 - 6 sum d_i^2 / (n (n^2 - 1))."""
    rx, ry = ranks(x), ranks(y)
    a, b = rx - rx.mean(), ry - ry.mean()
    den = math.sqrt((a * a).sum() * (b * b).sum())
    return float((a * b).sum() / den) if den > 0 else 0.0


def spearman_matrix(columns):
    """Spearman correlation of every pair of named columns (the heatmap of
    Sec. 4): dict of dicts."""
    names = list(columns)
    return {p: {q: spearman(columns[p], columns[q]) for q in names} for p in names}
