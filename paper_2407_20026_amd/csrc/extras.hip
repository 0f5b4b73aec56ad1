// Optimisation extras of the paper's examples: the displacement-violation penalty and the
// penalised material volume of the size optimisation (Sec. 3.3) with the pieces of their
// gradient, and the hat filter applied to nodal sensitivities (Sec. 3.1-3.2).
//
// Size objective: g = (1 + eps1 c) W with c = sum over nodes of max(0, |u_z| / u_max - 1) and
// W = sum over quads of A_e t_e + max(0, (t_min - t_e) / t_min).  dc/dp comes from the adjoint
// with dg/du = dc/du (sign(u_z) / u_max where the term is active); dW/dp from the element
// areas (k_volume_terms); k_size_combine forms eps1 W dc/dp + (1 + eps1 c) dW/dp per element
// term before the usual per-node gather.  All sums run in a fixed order.
#include "sso_internal.h"

namespace sso {
namespace {

constexpr int TPB = 256;

inline unsigned nblk(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

// Fixed-order workgroup sum of two values, returned in thread 0.
__device__ inline void wg_sum2(double v[2]) {
  __shared__ double lds[2][TPB / 64];
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 2; ++k) v[k] += __shfl_xor(v[k], off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < 2; ++k) lds[k][wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 2; ++k) {
      double s = lds[k][0];
      for (int w = 1; w < TPB / 64; ++w) s += lds[k][w];
      v[k] = s;
    }
}

// dc/du into dcdu (0 on constrained DOFs and on inactive nodes); per-workgroup partials of c
// (nodes) and W (the quads' shares w).
__global__ void __launch_bounds__(TPB)
k_size_terms(int n_nodes, int n_quads, const uint8_t* fixed, const double* u, double u_max,
             const double* w, double* dcdu, double* partials) {
  double v[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * TPB;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n_nodes; i += stride) {
    const double uz = u[6 * i + 2];
    const double a = fabs(uz) / u_max - 1.0;
    const bool active = a > 0.0;
    if (active) v[0] += a;
    for (int c = 0; c < 6; ++c) {
      const int64_t q = 6 * i + c;
      double g = 0.0;
      if (c == 2 && active && !fixed[q]) g = (uz > 0.0 ? 1.0 : (uz < 0.0 ? -1.0 : 0.0)) / u_max;
      dcdu[q] = g;
    }
  }
  for (int64_t e = blockIdx.x * (int64_t)TPB + threadIdx.x; e < n_quads; e += stride)
    v[1] += w[e];
  wg_sum2(v);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = v[0];
    partials[gridDim.x + blockIdx.x] = v[1];
  }
}

// One workgroup: out[0] = c, out[1] = W (partials of n workgroups, fixed order).
__global__ void __launch_bounds__(TPB) k_size_finish(const double* partials, int n, double* out) {
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += TPB) {
    v[0] += partials[i];
    v[1] += partials[n + i];
  }
  wg_sum2(v);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
  }
}

// Element terms of g: beams eps1 W dc; quads eps1 W dc + (1 + eps1 c) dW (sc = {c, W}).
__global__ void k_size_combine(int64_t n_beam_terms, int64_t n_quad_terms, double eps1,
                               const double* sc, const double* gw, double* gbeam,
                               double* gquad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double a = eps1 * sc[1], b = 1.0 + eps1 * sc[0];
  if (t < n_beam_terms) gbeam[t] = a * gbeam[t];
  if (t < n_quad_terms) gquad[t] = a * gquad[t] + b * gw[t];
}

// Hat filter: out[i] = sum_j w_ij g_j / sum_j w_ij, w_ij = max(0, r - |X_i - X_j|) over the n
// design nodes (ascending j; coordinates and sensitivities of a tile of j staged in LDS).
// Design node indices outside [0, n_nodes) set *err and are read as node 0.
__global__ void __launch_bounds__(TPB)
k_hat_filter(int n, const int32_t* nodes, int n_nodes, const double* xyz, const double* g,
             double r, double* out, unsigned* err) {
  __shared__ double tx[TPB], ty[TPB], tz[TPB], tg[TPB];
  const int i = blockIdx.x * TPB + threadIdx.x;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (i < n) {
    int ni = nodes ? nodes[i] : i;
    if (ni < 0 || ni >= n_nodes) {
      atomicOr(err, 1u);
      ni = 0;
    }
    xi = xyz[3 * (int64_t)ni];
    yi = xyz[3 * (int64_t)ni + 1];
    zi = xyz[3 * (int64_t)ni + 2];
  }
  double num = 0.0, den = 0.0;
  for (int j0 = 0; j0 < n; j0 += TPB) {
    const int j = j0 + threadIdx.x;
    if (j < n) {
      int nj = nodes ? nodes[j] : j;
      if (nj < 0 || nj >= n_nodes) nj = 0;
      tx[threadIdx.x] = xyz[3 * (int64_t)nj];
      ty[threadIdx.x] = xyz[3 * (int64_t)nj + 1];
      tz[threadIdx.x] = xyz[3 * (int64_t)nj + 2];
      tg[threadIdx.x] = g[j];
    }
    __syncthreads();
    const int lim = (n - j0) < TPB ? (n - j0) : TPB;
    for (int k = 0; k < lim; ++k) {
      const double dx = xi - tx[k], dy = yi - ty[k], dz = zi - tz[k];
      const double w = r - sqrt(dx * dx + dy * dy + dz * dz);
      if (w > 0.0) {
        num += w * tg[k];
        den += w;
      }
    }
    __syncthreads();
  }
  if (i < n) out[i] = num / den;
}

}  // namespace

hipError_t launch_size_terms(const Mesh& m, const double* u, double u_max, const double* w,
                             double* dcdu, double* partials, int max_wg, double* d_out,
                             hipStream_t s) {
  const int64_t n = m.n_nodes > m.n_quads ? m.n_nodes : m.n_quads;
  int g = (int)nblk(n, TPB);
  if (g > max_wg) g = max_wg;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_size_terms, dim3(g), dim3(TPB), 0, s, m.n_nodes, m.n_quads, m.fixed, u,
                     u_max, w, dcdu, partials);
  hipLaunchKernelGGL(k_size_finish, dim3(1), dim3(TPB), 0, s, partials, g, d_out);
  return hipGetLastError();
}

hipError_t launch_size_combine(const Mesh& m, double eps1, const double* sc, const double* gw,
                               double* gbeam, double* gquad, hipStream_t s) {
  const int64_t nb = 6 * (int64_t)m.n_beams, nq = 14 * (int64_t)m.n_quads;
  const int64_t n = nb > nq ? nb : nq;
  if (n)
    hipLaunchKernelGGL(k_size_combine, dim3(nblk(n, TPB)), dim3(TPB), 0, s, nb, nq, eps1, sc,
                       gw, gbeam, gquad);
  return hipGetLastError();
}

hipError_t launch_hat_filter(int n, const int32_t* nodes, const Mesh& m, const double* g,
                             double r, double* out, unsigned* err, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_hat_filter, dim3(nblk(n, TPB)), dim3(TPB), 0, s, n, nodes, m.n_nodes,
                       m.xyz, g, r, out, err);
  return hipGetLastError();
}

}  // namespace sso
