"""Oracle assembly: sparse pattern, scatter map, sort permutation, global K and load vector.

Paper: Sec. 2.2.1 -- element-to-global index maps give the row/column of every local stiffness
entry in K, and K is the sum of all element contributions, formed for all elements at once and
stored sparse.  Global DOF numbering is 6 * node + c with c in (ux, uy, uz, rx, ry, rz), the order
of the support and nodal-load vectors of the model-building API.

The element contribution list ("COO list") is element-major -- all beams, then all quads -- and
within an element the local matrix is listed row-major.  The pattern holds the 6x6 block (I, J)
iff I == J or some element contains both nodes; constrained DOFs stay in the pattern.

The scatter map is found here by a dictionary lookup of (row, col) -> CSR position, which is an
independent route from the sort that the device path uses.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import elements


def element_dofs(mesh):
    """Global DOF lists of beams [nb, 12] and quads [nq, 24]."""
    c6 = np.arange(6)
    bd = (6 * mesh.beam_nodes.astype(np.int64)[:, :, None] + c6).reshape(-1, 12)
    qd = (6 * mesh.quad_nodes.astype(np.int64)[:, :, None] + c6).reshape(-1, 24)
    return bd, qd


def block_pattern(mesh):
    """Sorted block columns of every block row (list of sorted lists)."""
    n = mesh.n_nodes
    cols = [set([i]) for i in range(n)]
    for conn in (mesh.beam_nodes, mesh.quad_nodes):
        for el in conn:
            for a in el:
                for b in el:
                    cols[int(a)].add(int(b))
    return [sorted(c) for c in cols]


def scalar_pattern(mesh):
    """Scalar CSR (row_ptr, col) of the 6-DOF-per-node pattern, int64 arrays."""
    bcols = block_pattern(mesh)
    row_ptr = [0]
    col = []
    for I, cs in enumerate(bcols):
        for a in range(6):
            for J in cs:
                for b in range(6):
                    col.append(6 * J + b)
            row_ptr.append(len(col))
    return np.array(row_ptr, np.int64), np.array(col, np.int64)


def coo_rows_cols(mesh):
    """(row, col) of every entry of the element-major, row-major COO list."""
    bd, qd = element_dofs(mesh)
    rows, cols = [], []
    for d in (bd, qd):
        n_loc = d.shape[1]
        rows.append(np.repeat(d, n_loc, axis=1).ravel())
        cols.append(np.tile(d, (1, n_loc)).ravel())
    return np.concatenate(rows), np.concatenate(cols)


def scatter_map(mesh, row_ptr, col):
    """S[k] = CSR position of COO entry k, by dictionary lookup."""
    pos = {}
    for r in range(len(row_ptr) - 1):
        for p in range(row_ptr[r], row_ptr[r + 1]):
            pos[(r, int(col[p]))] = p
    rows, cols = coo_rows_cols(mesh)
    return np.array([pos[(int(r), int(c))] for r, c in zip(rows, cols)], np.int64)


def sort_permutation(mesh):
    """perm = stable argsort of the COO keys row * n_dof + col (library sort)."""
    rows, cols = coo_rows_cols(mesh)
    keys = rows * mesh.n_dof + cols
    return np.argsort(keys, kind="stable")


def pattern(mesh):
    """Full pattern record: row_ptr, col, scatter S, perm and seg (all int64)."""
    row_ptr, col = scalar_pattern(mesh)
    S = scatter_map(mesh, row_ptr, col)
    perm = sort_permutation(mesh)
    # seg[s] = first position in perm of slot s; isolated diagonal blocks get empty segments
    counts = np.bincount(S, minlength=len(col))
    seg = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return dict(row_ptr=row_ptr, col=col, S=S, perm=perm, seg=seg)


def element_matrices(mesh, xyz=None, quad_t=None, quad_scale=None):
    """Global-DOF element matrices: beams [nb, 12, 12], quads [nq, 24, 24]."""
    xyz = mesh.xyz if xyz is None else xyz
    Kb = np.zeros((0, 12, 12))
    Kq = np.zeros((0, 24, 24))
    if mesh.n_beams:
        Kb = elements.beam_K(xyz[mesh.beam_nodes], mesh.beam_prop)
    if mesh.n_quads:
        prop = mesh.quad_prop.copy() if quad_t is None else mesh.quad_prop.astype(
            np.result_type(mesh.quad_prop, quad_t)).copy()
        if quad_t is not None:
            prop[:, 0] = quad_t
        scale = mesh.quad_scale if quad_scale is None else quad_scale
        Kq = elements.shell_K(xyz[mesh.quad_nodes], prop, scale)
    return Kb, Kq


def coo_values(mesh, xyz=None, quad_t=None, quad_scale=None):
    Kb, Kq = element_matrices(mesh, xyz, quad_t, quad_scale)
    return np.concatenate([Kb.reshape(-1), Kq.reshape(-1)])


def assemble(mesh, pat=None, xyz=None, quad_t=None, quad_scale=None):
    """Unconstrained global K (scipy CSR on the full pattern; values summed in COO order)."""
    pat = pattern(mesh) if pat is None else pat
    vals = coo_values(mesh, xyz, quad_t, quad_scale)
    data = np.zeros(len(pat["col"]), dtype=vals.dtype)
    np.add.at(data, pat["S"], vals)
    n = mesh.n_dof
    return sp.csr_matrix((data, pat["col"], pat["row_ptr"]), shape=(n, n))


def assemble_coo(mesh, xyz=None, quad_t=None, quad_scale=None):
    """Unconstrained global K as the plain sum K = sum_e P_e^T K_e P_e, formed by SciPy's
    duplicate summation of the (row, col, value) list (a library primitive, no dictionary).

    Same K as :func:`assemble` up to the order in which a slot's (at most four) contributions
    are added; used at sizes where the dictionary route of :func:`scatter_map` is too slow
    (hundreds of thousands of DOF)."""
    rows, cols = coo_rows_cols(mesh)
    vals = coo_values(mesh, xyz, quad_t, quad_scale)
    n = mesh.n_dof
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def load_vector(mesh, xyz=None, quad_t=None):
    """f = prescribed nodal loads - sum_e (gamma t_e + q) A_e / 4 on uz of each quad corner."""
    xyz = mesh.xyz if xyz is None else xyz
    t = mesh.quad_prop[:, 0] if quad_t is None else quad_t
    f = mesh.f_nodal.reshape(-1).astype(np.result_type(xyz, t))
    if mesh.n_quads and (mesh.unit_weight != 0.0 or mesh.surface_load != 0.0):
        fe = elements.shell_load(xyz[mesh.quad_nodes], t, mesh.unit_weight, mesh.surface_load)
        _, qd = element_dofs(mesh)
        np.add.at(f, qd.ravel(), fe.ravel())
    return f


def masked_system(mesh, K, f):
    """Support masking on the unchanged pattern: constrained d gets K[d, :] = K[:, d] = 0,
    K[d, d] = 1 and f[d] = 0.

    For zero prescribed displacements this gives the same u as the Lagrange-multiplier system of
    Sec. 2.2.1 (Eq. (2) with V u = 0) and as elimination of the constrained DOFs."""
    fixed = mesh.fixed.reshape(-1).astype(bool)
    K = K.tocsr()
    rows = np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))
    cols = K.indices
    data = K.data.copy()
    hit = fixed[rows] | fixed[cols]
    data[hit] = 0.0
    data[hit & (rows == cols)] = 1.0
    Km = sp.csr_matrix((data, cols.copy(), K.indptr.copy()), shape=K.shape)
    fm = np.where(fixed, 0.0, f)
    return Km, fm


# ---- local evaluations (one block row at a time) for spot checks at sizes where the global
# ---- pattern above would be too slow to build ---------------------------------------------

def incident(mesh, node):
    """Elements containing node, in element-list order: list of (kind, e, local index)."""
    out = []
    for kind, conn in (("beam", mesh.beam_nodes), ("quad", mesh.quad_nodes)):
        es, ls = np.nonzero(conn == node)
        for e, la in sorted(zip(es.tolist(), ls.tolist())):
            out.append((kind, e, la))
    return out


def block_row(mesh, I):
    """Sorted block columns of block row I (the diagonal block is always present)."""
    cols = {int(I)}
    for kind, e, _ in incident(mesh, I):
        conn = mesh.beam_nodes if kind == "beam" else mesh.quad_nodes
        cols.update(int(J) for J in conn[e])
    return sorted(cols)


def coo_index(mesh, kind, e, a, b):
    """Index of local entry (a, b) of element e in the element-major, row-major COO list."""
    if kind == "beam":
        return 144 * e + 12 * a + b
    return 144 * mesh.n_beams + 576 * e + 24 * a + b


def slot_contributions(mesh, row, col):
    """Ascending COO indices of the contributions to entry (row, col) of K."""
    I, ca = divmod(int(row), 6)
    J, cb = divmod(int(col), 6)
    ks = []
    for kind, e, la in incident(mesh, I):
        conn = mesh.beam_nodes if kind == "beam" else mesh.quad_nodes
        for lb, node in enumerate(conn[e]):
            if node == J:
                ks.append(coo_index(mesh, kind, e, 6 * la + ca, 6 * lb + cb))
    return sorted(ks)


def K_block_row(mesh, I):
    """Unconstrained block row I of K: dict J -> 6x6 block, summed in COO order."""
    out = {J: np.zeros((6, 6)) for J in block_row(mesh, I)}
    for kind, e, la in incident(mesh, I):
        if kind == "beam":
            Ke = elements.beam_K(mesh.xyz[mesh.beam_nodes[e:e + 1]], mesh.beam_prop[e:e + 1])[0]
            conn = mesh.beam_nodes[e]
        else:
            sc = None if mesh.quad_scale is None else mesh.quad_scale[e:e + 1]
            Ke = elements.shell_K(mesh.xyz[mesh.quad_nodes[e:e + 1]], mesh.quad_prop[e:e + 1],
                                  sc)[0]
            conn = mesh.quad_nodes[e]
        for lb, J in enumerate(conn):
            out[int(J)] += Ke[6 * la:6 * la + 6, 6 * lb:6 * lb + 6]
    return out


def apply_K_elementwise(mesh, u, chunk=10000):
    """K u (unconstrained) as the sum of element products, without forming the global K."""
    y = np.zeros(mesh.n_dof)
    bd, qd = element_dofs(mesh)
    for lo in range(0, mesh.n_beams, chunk):
        hi = min(mesh.n_beams, lo + chunk)
        Ke = elements.beam_K(mesh.xyz[mesh.beam_nodes[lo:hi]], mesh.beam_prop[lo:hi])
        np.add.at(y, bd[lo:hi].ravel(), (Ke @ u[bd[lo:hi]][:, :, None])[:, :, 0].ravel())
    for lo in range(0, mesh.n_quads, chunk):
        hi = min(mesh.n_quads, lo + chunk)
        sc = None if mesh.quad_scale is None else mesh.quad_scale[lo:hi]
        Ke = elements.shell_K(mesh.xyz[mesh.quad_nodes[lo:hi]], mesh.quad_prop[lo:hi], sc)
        np.add.at(y, qd[lo:hi].ravel(), (Ke @ u[qd[lo:hi]][:, :, None])[:, :, 0].ravel())
    return y
