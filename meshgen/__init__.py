"""Seeded synthetic structures: the shared input generators.

This module only lays out geometry, connectivity, material constants, support flags and
prescribed nodal forces.  It holds none of the method's arithmetic (no element stiffness, no
load lumping, no assembly, no solve): both the HIP path and the CPU oracle consume the arrays it
returns.

Every generator returns a ``Mesh`` whose arrays follow the C-ABI layout:

* ``xyz``          float64 [n_nodes, 3]   nodal coordinates (m)
* ``fixed``        uint8   [n_nodes, 6]   1 = fixed (ux, uy, uz, rx, ry, rz); the support flag
                                          vector of the model-building API (Sec. 2.2.1)
* ``f_nodal``      float64 [n_nodes, 6]   prescribed nodal forces / moments (N, N m)
* ``beam_nodes``   int32   [n_beams, 2]   end nodes i, j of each space-frame member
* ``beam_prop``    float64 [n_beams, 6]   E, G, A, Iy, Iz, J  (SI units)
* ``quad_nodes``   int32   [n_quads, 4]   corner nodes, counter-clockwise seen from the shell
                                          normal
* ``quad_prop``    float64 [n_quads, 5]   t, E, nu, kx, ky  (kx = ky = 1)
* ``quad_scale``   float64 [n_quads] or None   stiffness scale per quad (SIMP rho^3)
* ``unit_weight``  float    self-weight density of quads along -Z (N/m^3)
* ``surface_load`` float    uniform pressure along -Z on quad area (N/m^2)
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import numpy as np

PINNED = (1, 1, 1, 0, 0, 0)     # translations fixed, rotations free
CLAMPED = (1, 1, 1, 1, 1, 1)


@dataclass
class Mesh:
    xyz: np.ndarray
    fixed: np.ndarray
    f_nodal: np.ndarray
    beam_nodes: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    beam_prop: np.ndarray = field(default_factory=lambda: np.zeros((0, 6), np.float64))
    quad_nodes: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int32))
    quad_prop: np.ndarray = field(default_factory=lambda: np.zeros((0, 5), np.float64))
    quad_scale: np.ndarray | None = None
    unit_weight: float = 0.0
    surface_load: float = 0.0
    name: str = ""
    u_prescribed: np.ndarray | None = None   # [n_nodes, 6], used at fixed DOFs; None = zero

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_dof(self) -> int:
        return 6 * self.n_nodes

    @property
    def n_beams(self) -> int:
        return int(self.beam_nodes.shape[0])

    @property
    def n_quads(self) -> int:
        return int(self.quad_nodes.shape[0])

    def copy(self, **changes) -> "Mesh":
        m = replace(self, **changes)
        for k in ("xyz", "fixed", "f_nodal", "beam_nodes", "beam_prop", "quad_nodes",
                  "quad_prop"):
            if k not in changes:
                setattr(m, k, getattr(self, k).copy())
        if "quad_scale" not in changes and self.quad_scale is not None:
            m.quad_scale = self.quad_scale.copy()
        return m

    def validate(self) -> None:
        n = self.n_nodes
        assert self.xyz.dtype == np.float64 and self.xyz.shape == (n, 3)
        assert self.fixed.dtype == np.uint8 and self.fixed.shape == (n, 6)
        assert self.f_nodal.dtype == np.float64 and self.f_nodal.shape == (n, 6)
        assert self.beam_nodes.dtype == np.int32 and self.beam_nodes.shape[1] == 2
        assert self.beam_prop.dtype == np.float64 and self.beam_prop.shape == (self.n_beams, 6)
        assert self.quad_nodes.dtype == np.int32 and self.quad_nodes.shape[1] == 4
        assert self.quad_prop.dtype == np.float64 and self.quad_prop.shape == (self.n_quads, 5)
        if self.quad_scale is not None:
            assert self.quad_scale.dtype == np.float64 and self.quad_scale.shape == (self.n_quads,)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def grid_beams(n: int) -> np.ndarray:
    """Members along the grid lines of an n x n node grid (node id = i + n*j).

    All x-direction members first (row by row), then all y-direction members."""
    ids = np.arange(n * n, dtype=np.int64).reshape(n, n)          # [j, i]
    bx = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], 1)
    by = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], 1)
    return _c(np.concatenate([bx, by], 0), np.int32)


def grid_quads(m: int) -> np.ndarray:
    """Quads of an m x m element grid on (m+1)^2 nodes (node id = i + (m+1)*j), CCW from +Z."""
    n = m + 1
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    n0 = (i + n * j).ravel()
    return _c(np.stack([n0, n0 + 1, n0 + 1 + n, n0 + n], 1), np.int32)


def gridshell(n: int = 11, span: float = 10.0, rise: float = 2.0, noise: float = 0.05,
              seed: int = 0, E: float = 210e9, nu: float = 0.3, A: float = 1e-3,
              I: float = 1e-6, J: float = 2e-6, P: float = -10e3) -> Mesh:
    """Square grid-shell of space-frame members (Euler-Bernoulli 12-DOF beams).

    Node heights z = rise*sin(pi x/span)*sin(pi y/span) + N(0, noise^2); 4 corner nodes pinned;
    vertical nodal load P at every node.  Defaults: the 11 x 11 steel grid-shell, 220 members,
    726 DOF."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, span, n)
    y, x = np.meshgrid(s, s, indexing="ij")
    z = rise * np.sin(np.pi * x / span) * np.sin(np.pi * y / span)
    z = z + rng.normal(0.0, noise, size=z.shape)
    xyz = _c(np.stack([x.ravel(), y.ravel(), z.ravel()], 1), np.float64)
    nn = n * n
    fixed = np.zeros((nn, 6), np.uint8)
    for c in (0, n - 1, n * (n - 1), n * n - 1):
        fixed[c] = PINNED
    f = np.zeros((nn, 6))
    f[:, 2] = P
    beams = grid_beams(n)
    G = E / (2.0 * (1.0 + nu))
    prop = np.tile(np.array([E, G, A, I, I, J]), (beams.shape[0], 1))
    return Mesh(xyz=xyz, fixed=fixed, f_nodal=f, beam_nodes=beams, beam_prop=_c(prop, np.float64),
                name=f"gridshell{n}x{n}")


def arch_bridge(n_el: int, n_spans: int = 100, span: float = 30.0, rise: float = 10.0,
                E: float = 200e9, nu: float = 0.3, A: float = 0.05, Iy: float = 0.01,
                Iz: float = 0.01, J: float = 0.02, w: float = -100e3) -> Mesh:
    """The multi-span arch bridge of the paper's performance study: n_spans parabolic arches
    (span 30 m, rise 10 m) in the XZ plane, each cut into n_el equal-x beam elements, sharing
    their pier nodes; DOF = 6 (n_spans n_el + 1).  Piers pinned (translations) with the twist
    about the bridge axis also held, so the chain has no out-of-plane rigid rotation.
    Self-weight as downward nodal loads: w (N/m) times each node's tributary arc length.
    Section and load are not given by the paper: a steel box section is assumed."""
    n = n_spans * n_el + 1
    x = np.linspace(0.0, n_spans * span, n)
    s = (x % span) / span
    s[-1] = 1.0 if n_el else 0.0
    z = 4.0 * rise * s * (1.0 - s)
    z[::n_el] = 0.0
    xyz = _c(np.stack([x, np.zeros(n), z], 1), np.float64)
    fixed = np.zeros((n, 6), np.uint8)
    fixed[::n_el, :4] = 1
    seg = np.sqrt(np.diff(x) ** 2 + np.diff(z) ** 2)
    trib = np.zeros(n)
    trib[:-1] += 0.5 * seg
    trib[1:] += 0.5 * seg
    f = np.zeros((n, 6))
    f[:, 2] = w * trib
    beams = _c(np.stack([np.arange(n - 1), np.arange(1, n)], 1), np.int32)
    G = E / (2.0 * (1.0 + nu))
    prop = np.tile(np.array([E, G, A, Iy, Iz, J]), (n - 1, 1))
    return Mesh(xyz=xyz, fixed=fixed, f_nodal=f, beam_nodes=beams, beam_prop=_c(prop, np.float64),
                name=f"arch{n_spans}x{n_el}")


def bump_heights(x: np.ndarray, y: np.ndarray, L: float, rng: np.random.Generator,
                 n_bumps: int = 5, amp_max: float = 3.0) -> np.ndarray:
    """Sum of Gaussian bumps: amplitude ~ U[0, amp_max], centre ~ U[0, L]^2,
    width sigma ~ U[0.1 L, 0.25 L]; z = sum_k a_k exp(-|xy - c_k|^2 / (2 sigma_k^2))."""
    amps = rng.uniform(0.0, amp_max, n_bumps)
    cen = rng.uniform(0.0, L, (n_bumps, 2))
    sig = rng.uniform(0.1 * L, 0.25 * L, n_bumps)
    z = np.zeros_like(x)
    for a, (cx, cy), sg in zip(amps, cen, sig):
        z = z + a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sg * sg))
    return z


def shell(m: int = 60, L: float = 20.0, seed: int = 1, E: float = 30e9, nu: float = 0.2,
          t_range=(0.1, 0.3), unit_weight: float = 25e3, surface_load: float = 2e3,
          flat: bool = False) -> Mesh:
    """Continuous shell of m x m flat-shell quads on an L x L square.

    z from a seeded sum of 5 Gaussian bumps (amplitude 0-3 m), per-element thickness
    ~ U[t_range], all boundary nodes pinned, self-weight (unit_weight) + uniform surface load.
    Defaults: the 60 x 60 concrete shell, 3,721 nodes, 22,326 DOF."""
    rng = np.random.default_rng(seed)
    n = m + 1
    s = np.linspace(0.0, L, n)
    y, x = np.meshgrid(s, s, indexing="ij")
    z = np.zeros_like(x) if flat else bump_heights(x, y, L, rng)
    t = rng.uniform(t_range[0], t_range[1], m * m)
    xyz = _c(np.stack([x.ravel(), y.ravel(), z.ravel()], 1), np.float64)
    fixed = np.zeros((n * n, 6), np.uint8)
    ij = np.arange(n)
    bnd = np.unique(np.concatenate([ij, ij + n * (n - 1), ij * n, ij * n + n - 1]))
    fixed[bnd] = PINNED
    quads = grid_quads(m)
    prop = np.zeros((m * m, 5))
    prop[:, 0] = t
    prop[:, 1] = E
    prop[:, 2] = nu
    prop[:, 3] = 1.0
    prop[:, 4] = 1.0
    return Mesh(xyz=xyz, fixed=fixed, f_nodal=np.zeros((n * n, 6)), quad_nodes=quads,
                quad_prop=_c(prop, np.float64), unit_weight=float(unit_weight),
                surface_load=float(surface_load), name=f"shell{m}x{m}")


# Named workloads -------------------------------------------------------------------------

def grid_shell_11() -> Mesh:
    """11 x 11-node steel grid-shell, 220 members, 726 DOF, seed 0."""
    return gridshell(11, seed=0)


def shell_60() -> Mesh:
    """60 x 60 concrete shell, 22,326 DOF, seed 1."""
    return shell(60, seed=1)


def shell_300() -> Mesh:
    """300 x 300 concrete shell, 543,606 DOF, seed 2."""
    return shell(300, seed=2)


def served_request(i: int, base_seed: int = 10**6) -> Mesh:
    """One request of the mixed-size served stream: with probability 1/2 a grid-shell with
    n ~ U{8..60} nodes per side, else a quad shell with m ~ U{10..120} elements per side; all
    drawn from the per-request seed base_seed + i."""
    rng = np.random.default_rng(base_seed + i)
    if rng.integers(0, 2) == 0:
        n = int(rng.integers(8, 61))
        return gridshell(n, span=10.0, seed=int(rng.integers(0, 2**31)))
    m = int(rng.integers(10, 121))
    return shell(m, seed=int(rng.integers(0, 2**31)))


def density_field(n_quads: int, variant: int, base_seed: int = 4000,
                  lo: float = 0.01, hi: float = 1.0) -> np.ndarray:
    """Seeded per-element density rho ~ U[lo, hi] of one variant of the differentiable batch."""
    return np.random.default_rng(base_seed + variant).uniform(lo, hi, n_quads)
