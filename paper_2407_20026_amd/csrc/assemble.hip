// Assembly, support masking, loads and the block-Jacobi preconditioner.
//
// Sec. 2.2.1: K is the sum of all element matrices placed by their index maps; supports enter
// through Lagrange multipliers with V u = b.  The same displacement follows from masking: a
// constrained DOF d gets K[d, :] = K[:, d] = 0, K[d, d] = 1 and f[d] = 0, and with prescribed
// values b a free row's load loses K(row, d) b[d] (lifting; u = b is written on d after the
// solve), which keeps K symmetric positive definite and its pattern unchanged.
//
// Assembly is gather-based and deterministic: one thread per entry (slot, a, b) of a 6x6 block
// sums the slot's element contributions in ascending contribution id (= ascending element, then
// ascending scalar index), with no atomics, so K is bitwise reproducible.  An entry below the
// diagonal (block (I, J) with J < I, or a > b in a diagonal block) sums the contributions of its
// transposed entry, (b, a) of block (J, I), in the same order: the element matrices are
// symmetric only up to rounding, and this makes K bitwise symmetric, which lets the PCG
// products read a lower block as the transpose of its mirror.
#include "sso_internal.h"

namespace sso {
namespace {

inline unsigned nblk(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }


// K block values, row-major inside each 6x6 block, blocks in slot order.
__global__ void k_assemble(Mesh m, int64_t n_blocks, const int32_t* bsrow, const int32_t* bcol,
                           const int32_t* bseg, const int32_t* bperm, const int32_t* bsym,
                           const double* coo, double* K) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 36 * n_blocks) return;
  int64_t s = t / 36;
  int a = (int)(t % 36) / 6, b = (int)(t % 6);
  int I = bsrow[s], J = bcol[s];
  double v;
  if (m.fixed[6 * (int64_t)I + a] || m.fixed[6 * (int64_t)J + b]) {
    v = (I == J && a == b) ? 1.0 : 0.0;
  } else {
    // the upper triangle's entry whose value this one takes: itself, or its transpose (in the
    // value slot: block (J, I) for J < I, the slot itself otherwise)
    const bool low = J < I || (J == I && a > b);
    const int64_t su = bsym[2 * s + 1];
    const int ra = low ? b : a, rb = low ? a : b;
    v = 0.0;
    for (int p = bseg[su]; p < bseg[su + 1]; ++p) {
      BlockRef r = decode_block(bperm[p], m.n_beams);
      v += coo[coo_index(r, ra, rb, m.n_beams)];
    }
  }
  K[t] = v;
}

// f = f_nodal + sum over incident quads (ascending element) of -(gamma t + q) A / 4 on uz,
// masked.  The diagonal block slot of node I lists its incident elements in that order.
__global__ void k_loads(Mesh m, const int32_t* bdiag, const int32_t* bseg, const int32_t* bperm,
                        const double* qarea, double* f) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)m.n_nodes) return;
  int I = (int)(t / 6), c = (int)(t % 6);
  double v = m.f_nodal[t];
  if (c == 2 && (m.unit_weight != 0.0 || m.surface_load != 0.0)) {
    int s = bdiag[I];
    for (int p = bseg[s]; p < bseg[s + 1]; ++p) {
      BlockRef r = decode_block(bperm[p], m.n_beams);
      if (!r.quad) continue;
      double te = m.quad_prop[5 * (int64_t)r.e];
      v += -(m.unit_weight * te + m.surface_load) * qarea[r.e] / 4.0;
    }
  }
  f[t] = m.fixed[t] ? 0.0 : v;
}

// Prescribed support displacements b (Eq. 3 with b != 0) by lifting: the solve runs on
// u - b (b extended by 0 to the free DOFs), so f[t] = 0 on a constrained DOF (the masked row
// is the identity) and, on a free DOF t = 6 I + a, f[t] = fm[t] - sum over the slots of block
// row I (ascending) and components c of a constrained (J, c) of K(t, 6 J + c) b[6 J + c], with
// the unmasked entry summed from the element contributions in the assembly's order.  The
// solve keeps the constrained components at exactly 0 and solves K_ff u_f = f_f - K_fc b_c;
// k_apply_prescribed then writes u_c = b_c.
__global__ void k_lift(Mesh m, const int32_t* brow_ptr, const int32_t* bcol, const int32_t* bseg,
                       const int32_t* bperm, const double* coo, const double* fm, double* f) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)m.n_nodes) return;
  if (m.fixed[t]) {
    f[t] = 0.0;
    return;
  }
  const int I = (int)(t / 6), a = (int)(t % 6);
  double acc = 0.0;
  for (int s = brow_ptr[I]; s < brow_ptr[I + 1]; ++s) {
    const int64_t J = bcol[s];
    for (int c = 0; c < 6; ++c) {
      const int64_t d = 6 * J + c;
      if (!m.fixed[d] || m.u_presc[d] == 0.0) continue;
      double kv = 0.0;
      for (int p = bseg[s]; p < bseg[s + 1]; ++p) {
        const BlockRef r = decode_block(bperm[p], m.n_beams);
        kv += coo[coo_index(r, a, c, m.n_beams)];
      }
      acc += kv * m.u_presc[d];
    }
  }
  f[t] = fm[t] - acc;
}

__global__ void k_apply_prescribed(int64_t n, const uint8_t* fixed, const double* b, double* u) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n && fixed[t]) u[t] = b[t];
}

__global__ void k_mask_vector(int64_t n, const uint8_t* fixed, const double* in, double* out) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = fixed[t] ? 0.0 : in[t];
}

// Dinv_I = (K_II)^{-1} by Cholesky of the (masked, SPD) diagonal block, stored packed (upper
// triangle, dinv_index); entries (i, j) and (j, i) of W^T W are the same sum in the same order.
__global__ void k_block_jacobi(int n_nodes, const int32_t* bdiag, const double* K, double* Dinv,
                               float* Dinv32, unsigned* err) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  const double* A = K + 36 * (int64_t)bdiag[I];
  double L[6][6];
  bool ok = true;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L[i][j] = 0.0;
  for (int j = 0; j < 6; ++j) {
    double d = A[6 * j + j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0.0)) {
      ok = false;
      d = 1.0;
    }
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double v = A[6 * i + j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  if (!ok) atomicOr(err, ERR_DIAG);
  // W = L^{-1} (lower triangular), then Dinv = W^T W
  double W[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) W[i][j] = 0.0;
  for (int j = 0; j < 6; ++j) {
    W[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < 6; ++i) {
      double v = 0.0;
      for (int k = j; k < i; ++k) v -= L[i][k] * W[k][j];
      W[i][j] = v / L[i][i];
    }
  }
  double* out = Dinv + DINV_PACKED * (int64_t)I;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      double v = 0.0;
      for (int k = j; k < 6; ++k) v += W[k][i] * W[k][j];
      out[dinv_index(i, j)] = v;
      if (Dinv32) Dinv32[DINV_PACKED * (int64_t)I + dinv_index(i, j)] = (float)v;
    }
}

// Scalar CSR order of the block values (for read-back and parity checks).
__global__ void k_scalar_values(int n_nodes, const int32_t* brow_ptr, const double* K,
                                double* vals) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)n_nodes) return;
  int I = (int)(t / 6), a = (int)(t % 6);
  int rb = brow_ptr[I], nbc = brow_ptr[I + 1] - rb;
  int64_t rp = 36 * (int64_t)rb + 6 * (int64_t)a * nbc;
  for (int k = 0; k < nbc; ++k)
    for (int b = 0; b < 6; ++b) vals[rp + 6 * k + b] = K[36 * (int64_t)(rb + k) + 6 * a + b];
}

}  // namespace

hipError_t launch_assemble(const Mesh& m, const Pattern& pat, const double* coo, double* K,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(nblk(36 * pat.n_blocks, 256)), dim3(256), 0, s, m,
                     pat.n_blocks, pat.bsrow, pat.bcol, pat.bseg, pat.bperm, pat.bsym, coo,
                     K);
  return hipGetLastError();
}

hipError_t launch_loads(const Mesh& m, const Pattern& pat, const double* qarea, double* f,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_loads, dim3(nblk(6 * (int64_t)m.n_nodes, 256)), dim3(256), 0, s, m,
                     pat.bdiag, pat.bseg, pat.bperm, qarea, f);
  return hipGetLastError();
}

hipError_t launch_lift(const Mesh& m, const Pattern& pat, const double* coo, const double* fm,
                       double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_lift, dim3(nblk(6 * (int64_t)m.n_nodes, 256)), dim3(256), 0, s, m,
                     pat.brow_ptr, pat.bcol, pat.bseg, pat.bperm, coo, fm, f);
  return hipGetLastError();
}

hipError_t launch_apply_prescribed(const Mesh& m, double* u, hipStream_t s) {
  const int64_t n = 6 * (int64_t)m.n_nodes;
  hipLaunchKernelGGL(k_apply_prescribed, dim3(nblk(n, 256)), dim3(256), 0, s, n, m.fixed,
                     m.u_presc, u);
  return hipGetLastError();
}

hipError_t launch_mask_vector(const Mesh& m, const double* in, double* out, hipStream_t s) {
  int64_t n = 6 * (int64_t)m.n_nodes;
  hipLaunchKernelGGL(k_mask_vector, dim3(nblk(n, 256)), dim3(256), 0, s, n, m.fixed, in, out);
  return hipGetLastError();
}

hipError_t launch_block_jacobi(const Mesh& m, const Pattern& pat, const double* K, double* Dinv,
                               float* Dinv32, unsigned* d_err, hipStream_t s) {
  hipLaunchKernelGGL(k_block_jacobi, dim3(nblk(m.n_nodes, 128)), dim3(128), 0, s, m.n_nodes,
                     pat.bdiag, K, Dinv, Dinv32, d_err);
  return hipGetLastError();
}

hipError_t launch_scalar_values(const Mesh& m, const Pattern& pat, const double* K, double* vals,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_scalar_values, dim3(nblk(6 * (int64_t)m.n_nodes, 256)), dim3(256), 0, s,
                     m.n_nodes, pat.brow_ptr, K, vals);
  return hipGetLastError();
}

}  // namespace sso
