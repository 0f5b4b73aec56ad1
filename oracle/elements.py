"""Oracle element stiffness: 12-DOF space-frame member and 4-node flat shell.

Both routines are vectorised over elements and accept complex input so that the sensitivity
module can differentiate them by the complex-step method.  Branches test real parts only and
vector lengths are computed as sqrt(v . v), never with ``abs``, so every output is analytic in the
inputs.

Paper references: Sec. 2.2.1 -- the beam-column element of the model-building API takes
(E, G, Iy, Iz, J, A) and the two end nodes; the quad shell element is the MITC-4 formulation
(Dvorkin & Bathe 1984; Bathe 2006) whose attribute vector holds the 12 corner coordinates, t, E,
nu and two stiffness-modification coefficients.  The paper prints no element equations, so the
formulation below is the textbook one:

* beam: Euler-Bernoulli space frame, local axis e1 along the member, e2 = normalise(Z x e1)
  (e2 = Y for vertical members), e3 = e1 x e2, K = T^T k T with T = diag(R, R, R, R);
* shell: flat facet on the mean plane of the 4 corners -- bilinear Q4 membrane, Reissner-Mindlin
  plate with MITC4 assumed transverse shear, a displacement-form drilling penalty of factor
  1e-3 G t, a rigid offset from each corner to the mean plane, then K = T^T W^T k W T.
"""
from __future__ import annotations

import numpy as np

ALPHA_DRILL = 1.0e-3     # drilling penalty factor (times G t); fixed by specification
KAPPA_SHEAR = 5.0 / 6.0  # transverse shear correction factor
VERTICAL_TOL = 1.0e-6    # |Z x e1| below this: member treated as vertical

XI_N = np.array([-1.0, 1.0, 1.0, -1.0])   # natural coordinates of the 4 corners (CCW)
ETA_N = np.array([-1.0, -1.0, 1.0, 1.0])
_G = 1.0 / np.sqrt(3.0)
GAUSS_2x2 = [(-_G, -_G), (_G, -_G), (_G, _G), (-_G, _G)]   # all weights 1


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def _norm(a):
    return np.sqrt(_dot(a, a))


def _block_rotation(R, n_nodes):
    """T = diag(R, ..., R) with 2*n_nodes copies of the 3x3 rotation (rows = local axes)."""
    n = R.shape[0]
    T = np.zeros((n, 6 * n_nodes, 6 * n_nodes), dtype=R.dtype)
    for b in range(2 * n_nodes):
        T[:, 3 * b:3 * b + 3, 3 * b:3 * b + 3] = R
    return T


# ----------------------------------------------------------------------------- beam

def beam_frame(Xi, Xj):
    """Length and rotation R (rows e1, e2, e3) of members from end coordinates [n, 3]."""
    d = Xj - Xi
    L = _norm(d)
    e1 = d / L[:, None]
    zhat = np.zeros_like(e1)
    zhat[:, 2] = 1.0
    w = _cross(zhat, e1)
    nw = _norm(w)
    vertical = np.real(nw) < VERTICAL_TOL
    safe = np.where(vertical, 1.0, nw)
    yhat = np.zeros_like(e1)
    yhat[:, 1] = 1.0
    e2 = np.where(vertical[:, None], yhat, w / safe[:, None])
    e3 = _cross(e1, e2)
    return L, np.stack([e1, e2, e3], axis=1)


def beam_local_k(E, G, A, Iy, Iz, J, L):
    """Local 12x12 Euler-Bernoulli space-frame stiffness, DOFs (u v w tx ty tz) at i then j."""
    n = L.shape[0]
    dt = np.result_type(E, L)
    k = np.zeros((n, 12, 12), dtype=dt)
    L2, L3 = L * L, L * L * L

    def put(a, b, v):
        k[:, a, b] = v
        k[:, b, a] = v

    ea, gj = E * A / L, G * J / L
    put(0, 0, ea); put(6, 6, ea); put(0, 6, -ea)
    put(3, 3, gj); put(9, 9, gj); put(3, 9, -gj)
    # bending in the local x-y plane (v, tz), inertia Iz
    put(1, 1, 12 * E * Iz / L3); put(7, 7, 12 * E * Iz / L3); put(1, 7, -12 * E * Iz / L3)
    put(1, 5, 6 * E * Iz / L2); put(1, 11, 6 * E * Iz / L2)
    put(5, 7, -6 * E * Iz / L2); put(7, 11, -6 * E * Iz / L2)
    put(5, 5, 4 * E * Iz / L); put(11, 11, 4 * E * Iz / L); put(5, 11, 2 * E * Iz / L)
    # bending in the local x-z plane (w, ty), inertia Iy
    put(2, 2, 12 * E * Iy / L3); put(8, 8, 12 * E * Iy / L3); put(2, 8, -12 * E * Iy / L3)
    put(2, 4, -6 * E * Iy / L2); put(2, 10, -6 * E * Iy / L2)
    put(4, 8, 6 * E * Iy / L2); put(8, 10, 6 * E * Iy / L2)
    put(4, 4, 4 * E * Iy / L); put(10, 10, 4 * E * Iy / L); put(4, 10, 2 * E * Iy / L)
    return k


def beam_K(X, prop, scale=None):
    """Global 12x12 stiffness of members.  X [n, 2, 3]; prop [n, 6] = (E, G, A, Iy, Iz, J)."""
    L, R = beam_frame(X[:, 0], X[:, 1])
    E, G, A, Iy, Iz, J = (prop[:, c] for c in range(6))
    k = beam_local_k(E, G, A, Iy, Iz, J, L)
    T = _block_rotation(R, 2)
    K = np.swapaxes(T, 1, 2) @ k @ T
    if scale is not None:
        K = K * scale[:, None, None]
    return K


# ----------------------------------------------------------------------------- shell

def shape_functions(xi, eta):
    """Bilinear N_i and their natural derivatives at one point (arrays of 4)."""
    N = 0.25 * (1 + xi * XI_N) * (1 + eta * ETA_N)
    dxi = 0.25 * XI_N * (1 + eta * ETA_N)
    deta = 0.25 * ETA_N * (1 + xi * XI_N)
    return N, dxi, deta


def shell_frame(X):
    """Mean-plane frame of quads X [n, 4, 3].

    e3 = normalise(d13 x d24) (diagonals), e1 = the xi-midline direction projected on the mean
    plane, e2 = e3 x e1.  Returns R (rows e1, e2, e3), local in-plane coordinates x, y [n, 4],
    the offsets h [n, 4] of the corners from the mean plane, and the area A = |d13 x d24| / 2."""
    c = X.mean(axis=1)
    d13 = X[:, 2] - X[:, 0]
    d24 = X[:, 3] - X[:, 1]
    nv = _cross(d13, d24)
    nn = _norm(nv)
    e3 = nv / nn[:, None]
    a = 0.5 * (X[:, 1] + X[:, 2] - X[:, 0] - X[:, 3])
    ap = a - _dot(a, e3)[:, None] * e3
    e1 = ap / _norm(ap)[:, None]
    e2 = _cross(e3, e1)
    rel = X - c[:, None, :]
    x = _dot(rel, e1[:, None, :])
    y = _dot(rel, e2[:, None, :])
    h = _dot(rel, e3[:, None, :])
    return np.stack([e1, e2, e3], axis=1), x, y, h, 0.5 * nn


def _jacobian(x, y, xi, eta):
    _, dxi, deta = shape_functions(xi, eta)
    J11, J12 = x @ dxi, y @ dxi
    J21, J22 = x @ deta, y @ deta
    det = J11 * J22 - J12 * J21
    Jinv = np.stack([np.stack([J22, -J12], -1), np.stack([-J21, J11], -1)], -2) / det[:, None, None]
    return det, Jinv


def _covariant_shear_row(x, y, xi_t, eta_t, direction):
    """Row (over the 24 local DOFs) of the covariant transverse shear strain at a tying point.

    gamma_r = w,r + beta_x x,r + beta_y y,r with r = xi (direction 0) or eta (direction 1),
    beta_x = theta_y, beta_y = -theta_x, every field interpolated bilinearly."""
    N, dxi, deta = shape_functions(xi_t, eta_t)
    dr = dxi if direction == 0 else deta
    x_r = x @ dr
    y_r = y @ dr
    row = np.zeros((x.shape[0], 24), dtype=x.dtype)
    for i in range(4):
        row[:, 6 * i + 2] = dr[i]
        row[:, 6 * i + 4] = N[i] * x_r          # beta_x = theta_y
        row[:, 6 * i + 3] = -N[i] * y_r         # beta_y = -theta_x
    return row


def shell_local_parts(x, y, t, E, nu):
    """Local 24x24 stiffness parts (membrane, bending, shear, drilling) of flat quads.

    x, y [n, 4] local corner coordinates; t, E, nu [n].  2x2 Gauss quadrature throughout."""
    n = x.shape[0]
    dt = np.result_type(x, t, E)
    G = E / (2 * (1 + nu))
    C = np.zeros((n, 3, 3), dtype=np.result_type(nu, float))
    C[:, 0, 0] = 1; C[:, 1, 1] = 1
    C[:, 0, 1] = nu; C[:, 1, 0] = nu
    C[:, 2, 2] = (1 - nu) / 2
    Dm = (E * t / (1 - nu * nu))[:, None, None] * C
    Db = (E * t ** 3 / (12 * (1 - nu * nu)))[:, None, None] * C
    ks = KAPPA_SHEAR * G * t
    kd = ALPHA_DRILL * G * t
    # MITC4 tying points: A (0,+1), C (0,-1) carry gamma_xi; B (-1,0), D (+1,0) carry gamma_eta
    gA = _covariant_shear_row(x, y, 0.0, 1.0, 0)
    gC = _covariant_shear_row(x, y, 0.0, -1.0, 0)
    gB = _covariant_shear_row(x, y, -1.0, 0.0, 1)
    gD = _covariant_shear_row(x, y, 1.0, 0.0, 1)
    Km = np.zeros((n, 24, 24), dtype=dt)
    Kb = np.zeros_like(Km)
    Ks = np.zeros_like(Km)
    Kd = np.zeros_like(Km)
    for xi, eta in GAUSS_2x2:
        det, Jinv = _jacobian(x, y, xi, eta)
        N, dxi, deta = shape_functions(xi, eta)
        dNdx = Jinv[:, 0, 0, None] * dxi + Jinv[:, 0, 1, None] * deta    # [n, 4]
        dNdy = Jinv[:, 1, 0, None] * dxi + Jinv[:, 1, 1, None] * deta
        Bm = np.zeros((n, 3, 24), dtype=dt)
        Bb = np.zeros((n, 3, 24), dtype=dt)
        bd = np.zeros((n, 24), dtype=dt)
        for i in range(4):
            u, v, th_x, th_y, th_z = 6 * i, 6 * i + 1, 6 * i + 3, 6 * i + 4, 6 * i + 5
            Bm[:, 0, u] = dNdx[:, i]
            Bm[:, 1, v] = dNdy[:, i]
            Bm[:, 2, u] = dNdy[:, i]
            Bm[:, 2, v] = dNdx[:, i]
            # curvatures of beta = (theta_y, -theta_x)
            Bb[:, 0, th_y] = dNdx[:, i]
            Bb[:, 1, th_x] = -dNdy[:, i]
            Bb[:, 2, th_y] = dNdy[:, i]
            Bb[:, 2, th_x] = -dNdx[:, i]
            # drilling: theta_z - (v,x - u,y)/2
            bd[:, th_z] = N[i]
            bd[:, v] = -0.5 * dNdx[:, i]
            bd[:, u] = 0.5 * dNdy[:, i]
        g_xi = 0.5 * (1 + eta) * gA + 0.5 * (1 - eta) * gC
        g_eta = 0.5 * (1 + xi) * gD + 0.5 * (1 - xi) * gB
        Bs = Jinv @ np.stack([g_xi, g_eta], axis=1)
        w = det[:, None, None]
        Km += w * (np.swapaxes(Bm, 1, 2) @ Dm @ Bm)
        Kb += w * (np.swapaxes(Bb, 1, 2) @ Db @ Bb)
        Ks += (w * ks[:, None, None]) * (np.swapaxes(Bs, 1, 2) @ Bs)
        Kd += (w * kd[:, None, None]) * bd[:, :, None] * bd[:, None, :]
    return Km, Kb, Ks, Kd


def min_gauss_detJ(x, y):
    """Smallest Jacobian determinant over the 2x2 Gauss points (real part)."""
    return np.min(np.stack([np.real(_jacobian(x, y, xi, eta)[0]) for xi, eta in GAUSS_2x2]),
                  axis=0)


def warp_matrix(h):
    """W: u_i <- u_i - h_i theta_y,i ; v_i <- v_i + h_i theta_x,i (rigid offset to mean plane)."""
    n = h.shape[0]
    W = np.zeros((n, 24, 24), dtype=h.dtype)
    W[:, np.arange(24), np.arange(24)] = 1.0
    for i in range(4):
        W[:, 6 * i + 0, 6 * i + 4] = -h[:, i]
        W[:, 6 * i + 1, 6 * i + 3] = h[:, i]
    return W


def shell_K_parts(X, prop, scale=None):
    """Global 24x24 stiffness parts (membrane, bending, shear, drilling) of quads.

    X [n, 4, 3]; prop [n, 5] = (t, E, nu, kx, ky).  Returns a list of 4 arrays [n, 24, 24] whose
    sum is K_e = s T^T W^T k W T."""
    R, x, y, h, _ = shell_frame(X)
    t, E, nu = prop[:, 0], prop[:, 1], prop[:, 2]
    parts = shell_local_parts(x, y, t, E, nu)
    W = warp_matrix(h)
    T = _block_rotation(R, 4)
    WT = W @ T
    out = []
    for k in parts:
        K = np.swapaxes(WT, 1, 2) @ k @ WT
        if scale is not None:
            K = K * scale[:, None, None]
        out.append(K)
    return out


def shell_K(X, prop, scale=None):
    Km, Kb, Ks, Kd = shell_K_parts(X, prop, scale)
    return Km + Kb + Ks + Kd


def shell_area(X):
    """Element area used for surface and self-weight loads: |d13 x d24| / 2."""
    return shell_frame(X)[4]


def shell_load(X, t, unit_weight, surface_load):
    """Consistent-by-lumping vertical load of quads: -(gamma t + q) A / 4 on uz of each corner.

    Returns f_e [n, 24] in global DOFs."""
    A = shell_area(X)
    fz = -(unit_weight * t + surface_load) * A / 4.0
    f = np.zeros((X.shape[0], 24), dtype=fz.dtype)
    for i in range(4):
        f[:, 6 * i + 2] = fz
    return f
