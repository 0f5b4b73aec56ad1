"""Small hand-built structures for the oracle pins (closed-form cases).

Only geometry, connectivity, supports and loads are laid out here; no element arithmetic."""
import numpy as np

from meshgen import Mesh, grid_quads


def cantilever(direction, L=2.0, n_el=1, E=200e9, nu=0.3, A=3e-3, Iy=2e-6, Iz=5e-6, J=4e-6,
               origin=(0.3, -0.2, 0.5)):
    d = np.asarray(direction, float)
    d = d / np.sqrt(d @ d)
    s = np.linspace(0.0, L, n_el + 1)
    xyz = np.ascontiguousarray(np.asarray(origin)[None, :] + s[:, None] * d[None, :])
    n = n_el + 1
    fixed = np.zeros((n, 6), np.uint8)
    fixed[0] = 1
    bn = np.stack([np.arange(n_el), np.arange(1, n)], 1).astype(np.int32)
    G = E / (2 * (1 + nu))
    prop = np.tile([E, G, A, Iy, Iz, J], (n_el, 1)).astype(np.float64)
    return Mesh(xyz=xyz, fixed=fixed, f_nodal=np.zeros((n, 6)), beam_nodes=bn, beam_prop=prop)


def plate(m, a=1.0, t=0.01, E=1.0e9, nu=0.3, q=0.0, jitter=0.0, seed=0, z=None):
    """Flat (z = 0 unless given) m x m quad plate on [0, a]^2; interior nodes optionally
    jittered in-plane; no supports; surface load q."""
    n = m + 1
    s = np.linspace(0.0, a, n)
    y, x = np.meshgrid(s, s, indexing="ij")
    x, y = x.ravel().copy(), y.ravel().copy()
    if jitter:
        rng = np.random.default_rng(seed)
        interior = (x > 0) & (x < a) & (y > 0) & (y < a)
        h = a / m
        x[interior] += rng.uniform(-jitter, jitter, interior.sum()) * h
        y[interior] += rng.uniform(-jitter, jitter, interior.sum()) * h
    zz = np.zeros_like(x) if z is None else z(x, y)
    xyz = np.ascontiguousarray(np.stack([x, y, zz], 1))
    prop = np.tile([t, E, nu, 1.0, 1.0], (m * m, 1)).astype(np.float64)
    return Mesh(xyz=xyz, fixed=np.zeros((n * n, 6), np.uint8), f_nodal=np.zeros((n * n, 6)),
                quad_nodes=grid_quads(m), quad_prop=prop, surface_load=float(q))


def boundary_nodes(m):
    n = m + 1
    ij = np.arange(n)
    return np.unique(np.concatenate([ij, ij + n * (n - 1), ij * n, ij * n + n - 1]))


def rigid_body_modes(xyz):
    """6 rigid-body displacement vectors [6, 6 n]: 3 translations, 3 rotations about the axes
    through the origin (u = w x X, theta = w)."""
    n = xyz.shape[0]
    modes = np.zeros((6, n, 6))
    for k in range(3):
        modes[k, :, k] = 1.0
        w = np.zeros(3)
        w[k] = 1.0
        modes[3 + k, :, :3] = np.cross(w[None, :], xyz)
        modes[3 + k, :, 3:] = w
    return modes.reshape(6, -1)


def solve_prescribed(K, f, prescribed):
    """Solve K u = f with u[d] = value for d in prescribed (dict), dense; returns full u."""
    K = K.toarray() if hasattr(K, "toarray") else K
    n = K.shape[0]
    c = np.array(sorted(prescribed), dtype=np.int64)
    uc = np.array([prescribed[i] for i in c])
    fr = np.setdiff1d(np.arange(n), c)
    u = np.zeros(n)
    u[c] = uc
    u[fr] = np.linalg.solve(K[np.ix_(fr, fr)], f[fr] - K[np.ix_(fr, c)] @ uc)
    return u
