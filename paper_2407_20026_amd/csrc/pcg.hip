// Block-Jacobi preconditioned conjugate gradients on the masked K (BSR, 6x6 blocks).
//
// The paper solves K u = f (Eq. 1, with the supports of Eqs. 2-3) with direct solvers
// (Sec. 2.2.2).  On the GPU the solve is a bandwidth-bound iteration instead, in one of two
// forms: the standard recurrences (two kernels per iteration, below) or the single-reduction
// recurrences of Chronopoulos and Gear (one kernel per iteration, k_cg1_*, further down).
// Standard iteration j:
//   k_spmv_dir : finish r_j^T z_j and r_j^T r_j from the previous kernel's per-workgroup
//                partials, test convergence, beta_j = rz_j / rz_{j-1}; p_j = z_j + beta_j p_{j-1}
//                (own rows stored, neighbour rows formed on the fly), Ap_j = K p_j, partial
//                p_j^T A p_j
//   k_update   : finish p_j^T A p_j, alpha_j = rz_j / pAp_j; x += alpha p, r -= alpha Ap,
//                z = Dinv r, partials r^T z and r^T r
// Every workgroup sums the previous kernel's partials itself, in the same fixed order, so all
// workgroups take identical decisions and no atomics or device-scope fences are needed; the
// kernel boundary makes the partials visible.  Workgroup 0 records the scalars the host polls.
// Once the state says done, later kernels return at entry, so the host launches iterations in
// chunks and polls between chunks.  Every reduction is deterministic.
//
// Thread layouts: the SpMV kernels give 18 lanes to a block row, each lane reading one 16-byte
// piece of every 6x6 block, so one load instruction covers a whole 288-byte block; the vector
// kernels give 6 lanes to a node.  All kernels stride over the rows with a fixed number of
// workgroups.  The recursively updated residual can drift below the true one (rounding); the
// FP64 driver therefore recomputes the true residual after convergence (row sums in
// double-double, k_residual) and, if it is above the target, solves for a correction (a few
// steps of iterative refinement).
#include <cmath>

#include "sso_internal.h"

namespace sso {
namespace {

constexpr int MAX_TPB = 384;
constexpr int MAX_WAVES = MAX_TPB / 64;
// Workgroups of a PCG launch at most (grid-stride beyond); see choose_wg.
constexpr int PCG_MAX_WG = 1024;

inline unsigned nblk(int64_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Where a workgroup of a (possibly multi-problem) PCG launch works: its problem's descriptor,
// its index among that problem's workgroups and their number.
template <class Desc>
struct WgOf {
  const Desc* d;
  int lb, ng;
};

template <class Desc>
__device__ inline WgOf<Desc> wg_of(const Desc* __restrict__ D,
                                   const int32_t* __restrict__ wg_prob) {
  WgOf<Desc> w;
  w.d = D + (wg_prob ? wg_prob[blockIdx.x] : 0);
  w.lb = (int)blockIdx.x - w.d->wg_base;
  w.ng = w.d->n_wg;
  return w;
}

template <class T>
using Wg = WgOf<PcgDesc<T>>;

// Cross-lane moves through DPP, register to register in a few cycles, where a shuffle would be
// a round trip through the LDS crossbar.  CTRL is the DPP control word: quad_perm 0x00-0xff,
// row_ror:n 0x120 + n.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((int)b, lane);
  const unsigned hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Sum over the 64 lanes of a wave, the same value in every lane: each quad by two quad_perm
// exchanges, each 16-lane row by rotations of 4 and 8 (lane 16r then holds its row's sum), and
// the four row sums in a fixed order.
template <class A>
__device__ __forceinline__ A wave_sum(A v) {
  v += dpp_move<0xb1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4e>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x124>(v);   // row_ror:4
  v += dpp_move<0x128>(v);   // row_ror:8
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Fixed-order workgroup sum of NV values; the result is returned to every thread.  TAG gives
// a call site its own LDS array; LAST (the array is not written again before the kernel ends
// or before a barrier) drops the trailing barrier that protects the array's reuse.  Called by
// every thread of the workgroup (full waves).
template <int NV, class A, int TAG = 0, bool LAST = false>
__device__ inline void block_sum(A v[NV]) {
  __shared__ A lds[NV][MAX_WAVES];
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
    for (int k = 0; k < NV; ++k) lds[k][wave] = v[k];
  __syncthreads();
  for (int k = 0; k < NV; ++k) {
    A s = lds[k][0];
    for (int w = 1; w < nw; ++w) s += lds[k][w];
    v[k] = s;
  }
  if (!LAST) __syncthreads();
}

// Sum of NV arrays of n per-workgroup partials (array k at partials + k * n), fixed order.
template <int NV>
__device__ inline void finish_partials(const double* partials, int n, double tot[NV]) {
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[k * n + i];
    tot[k] = s;
  }
  block_sum<NV, double>(tot);
}

template <int NV, class A>
__device__ inline void write_partials(const A v[NV], double* partials, int lb, int ng) {
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) partials[k * ng + lb] = (double)v[k];
}

template <int NV, class A>
__device__ inline void write_partials(const A v[NV], double* partials) {
  write_partials<NV, A>(v, partials, blockIdx.x, gridDim.x);
}

// ---- vector kernels: 6 consecutive lanes per node, 64 nodes per workgroup pass -----------

constexpr int VEC_NODES = MAX_TPB / 6;   // 64
static_assert(VEC_NODES == DINV_GROUP, "a vector pass covers one group of packed inverses");

struct RowMap {
  int lr, a, I;
  bool valid;
};

__device__ inline RowMap row_map_at(int group, int n_nodes) {
  RowMap m;
  m.lr = threadIdx.x / 6;
  m.a = threadIdx.x - 6 * m.lr;
  m.I = group * VEC_NODES + m.lr;
  m.valid = (m.lr < VEC_NODES) && (m.I < n_nodes);
  return m;
}

// The packed block-Jacobi inverses of a group of 64 nodes (21 x 64 values, contiguous) are
// loaded by the whole workgroup in 16-byte pieces -- each thread at most two, no bound test
// (the array is padded to whole groups) -- and staged in LDS, where the 6 lanes of each node read
// their rows.  Against every lane loading its own row of a full 6 x 6 block this reads 21 of 36
// values per node from HBM, in coalesced loads.
template <class T>
struct DinvChunk {
  static constexpr int PER = 16 / sizeof(T);                            // values per piece
  static constexpr int PIECES = DINV_PACKED * DINV_GROUP / PER;         // pieces per group
  static constexpr int PER_THREAD = (PIECES + MAX_TPB - 1) / MAX_TPB;
  using V = int4;
  V v[PER_THREAD];
};

template <class T>
__device__ inline DinvChunk<T> dinv_load(const T* __restrict__ Dinv, int group) {
  using C = DinvChunk<T>;
  C c;
  const typename C::V* src =
      reinterpret_cast<const typename C::V*>(Dinv + (int64_t)DINV_PACKED * DINV_GROUP * group);
  for (int k = 0; k < C::PER_THREAD; ++k) {
    const int i = (int)threadIdx.x + k * MAX_TPB;
    if (i < C::PIECES) c.v[k] = src[i];
  }
  return c;
}

template <class T>
__device__ inline void dinv_stage(const DinvChunk<T>& c, T* dl) {
  using C = DinvChunk<T>;
  typename C::V* dst = reinterpret_cast<typename C::V*>(dl);
  for (int k = 0; k < C::PER_THREAD; ++k) {
    const int i = (int)threadIdx.x + k * MAX_TPB;
    if (i < C::PIECES) dst[i] = c.v[k];
  }
}

// z = Dinv r for the node of this lane: row a of the node's inverse (staged in LDS at dl) applied
// to its r values (staged at rs), in the order of the row: (0, 1), (2, 3), (4, 5).
template <class T>
__device__ inline T apply_dinv(const T* dl, const T* rs, int a, int lr) {
  const T* dn = dl + DINV_PACKED * lr;
  const T* rr = rs + 6 * lr;
  T z = 0;
  for (int h = 0; h < 3; ++h)
    z += dn[dinv_index(a, 2 * h)] * rr[2 * h] + dn[dinv_index(a, 2 * h + 1)] * rr[2 * h + 1];
  return z;
}

// A store of a vector entry that the iteration writes: streaming (non-temporal) for problems
// whose K alone outgrows the caches (nothing written is read again before it would have been
// evicted), plain otherwise (small problems read it back from cache).
template <class T>
__device__ __forceinline__ void put(T* p, T v, int streaming) {
  if (streaming)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Row a of a node's packed block-Jacobi inverse, applied to the node's six values.
template <class T>
struct DinvRow {
  T d[6];
  __device__ inline T apply(const T* v) const {
    T z = 0;
    for (int h = 0; h < 3; ++h) z += d[2 * h] * v[2 * h] + d[2 * h + 1] * v[2 * h + 1];
    return z;
  }
};

template <class T>
__device__ inline DinvRow<T> dinv_row(const T* Dinv, int I, int a) {
  const T* dn = Dinv + DINV_PACKED * (int64_t)I;
  DinvRow<T> R;
  for (int b = 0; b < 6; ++b) R.d[b] = dn[dinv_index(a, b)];
  return R;
}

// ---- SpMV layout: 18 lanes per block row, 3 block rows per wavefront ----------------------
// Lane l of a row group owns entries (a, b..b+1) of every 6x6 block, a = l / 3, b = 2 (l % 3),
// so the 18 lanes read each 288-byte block with one contiguous 16-byte load each.

constexpr int ROW_LANES = 18;
constexpr int ROWS_PER_WAVE = 3;
constexpr int ROWS_PER_WG = ROWS_PER_WAVE * (MAX_TPB / 64);   // 18

struct SpLane {
  int lane, g, l, a, b;
  bool ok;
};

__device__ inline SpLane sp_lane() {
  SpLane L;
  L.lane = threadIdx.x & 63;
  L.g = L.lane / ROW_LANES;
  L.l = L.lane - ROW_LANES * L.g;
  L.a = L.l / 3;
  L.b = 2 * (L.l - 3 * L.a);
  L.ok = L.g < ROWS_PER_WAVE;
  return L;
}

// sum over the block row of K[s][a][b..b+1] . v[6 J + b..b+1], with v = x (DIR false) or
// v = x + beta p (DIR true, the search direction formed on the fly).  Unrolled by 3 blocks so
// the column indices of a step are loaded before the values that depend on them.
template <class T, bool DIR>
__device__ inline T row_product(const int32_t* __restrict__ brow_ptr,
                                const int32_t* __restrict__ bcol, const T* __restrict__ K,
                                const T* __restrict__ x, const T* __restrict__ p, T beta, int I,
                                int a, int b) {
  using V = typename Vec2<T>::type;
  const int rb = brow_ptr[I], re = brow_ptr[I + 1];
  const int off = 6 * a + b;
  T acc = 0;
  int s = rb;
  for (; s + 3 <= re; s += 3) {
    const int64_t J0 = bcol[s], J1 = bcol[s + 1], J2 = bcol[s + 2];
    const V k0 = *reinterpret_cast<const V*>(K + 36 * (int64_t)s + off);
    const V k1 = *reinterpret_cast<const V*>(K + 36 * (int64_t)(s + 1) + off);
    const V k2 = *reinterpret_cast<const V*>(K + 36 * (int64_t)(s + 2) + off);
    V x0 = *reinterpret_cast<const V*>(x + 6 * J0 + b);
    V x1 = *reinterpret_cast<const V*>(x + 6 * J1 + b);
    V x2 = *reinterpret_cast<const V*>(x + 6 * J2 + b);
    if (DIR) {
      const V p0 = *reinterpret_cast<const V*>(p + 6 * J0 + b);
      const V p1 = *reinterpret_cast<const V*>(p + 6 * J1 + b);
      const V p2 = *reinterpret_cast<const V*>(p + 6 * J2 + b);
      x0.x = x0.x + beta * p0.x; x0.y = x0.y + beta * p0.y;
      x1.x = x1.x + beta * p1.x; x1.y = x1.y + beta * p1.y;
      x2.x = x2.x + beta * p2.x; x2.y = x2.y + beta * p2.y;
    }
    acc += k0.x * x0.x + k0.y * x0.y;
    acc += k1.x * x1.x + k1.y * x1.y;
    acc += k2.x * x2.x + k2.y * x2.y;
  }
  for (; s < re; ++s) {
    const int64_t J = bcol[s];
    const V kv = *reinterpret_cast<const V*>(K + 36 * (int64_t)s + off);
    V xv = *reinterpret_cast<const V*>(x + 6 * J + b);
    if (DIR) {
      const V pv = *reinterpret_cast<const V*>(p + 6 * J + b);
      xv.x = xv.x + beta * pv.x; xv.y = xv.y + beta * pv.y;
    }
    acc += kv.x * xv.x + kv.y * xv.y;
  }
  return acc;
}

// Row total in the first lane (l % 3 == 0) of each 3-lane set, fixed order; the next two
// lanes' values come by one and two wave_shl:1 moves (lane i reads lane i + 1).  Every lane of
// the wave must be active.
template <class T>
__device__ inline T sum3(T acc) {
  const T t1 = dpp_move<0x130>(acc);
  const T t2 = dpp_move<0x130>(t1);
  return acc + t1 + t2;
}

// Pointers into global memory: the kernels take their operands from descriptors read from
// memory, so the compiler sees generic pointers and emits flat loads, whose completion it can
// only wait for together with every other memory and LDS operation in flight.  Through these
// it emits global loads and waits for exactly the loads a value needs.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}
template <class T>
struct Native2 {
  typedef T type __attribute__((ext_vector_type(2)));
};
template <class V, class T>
__device__ __forceinline__ V load2(gptr<T> p) {
  typedef typename Native2<T>::type N;
  const N v = *(const __attribute__((address_space(1))) N*)p;
  V r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

// sum over the block row of K[s][a][b..b+1] . z and . p (two accumulators, so the products do
// not wait for beta): the direction's product is K p_new = Kz + beta Kp.  NB blocks per step; a
// step issues its K values and gathers together with the block columns of the next step, so a
// step costs one round trip to memory instead of two (the columns, then the gathers that need
// them).  Indices past the row's end are clamped to its last block and their products not
// added, so every NB gives the products of one block after another, in that order (bitwise the
// same sums as row_product2 below, the two-block form without the clamping, which measured
// faster where bandwidth bounds the pair).
template <class T, int NB>
__device__ inline void row_product_nb(int rb, int re, const int32_t* __restrict__ bcol_,
                                      const T* __restrict__ K_, const T* __restrict__ z_,
                                      const T* __restrict__ p_, int a, int b, T& az, T& ap) {
  using V = typename Vec2<T>::type;
  const gptr<int32_t> bcol = as_global(bcol_);
  const gptr<T> K = as_global(K_);
  const gptr<T> z = as_global(z_);
  const gptr<T> p = as_global(p_);
  const int off = 6 * a + b;
  const int last = re - 1;
  T sz = 0, sp = 0;
  int s = rb;
  if (s < re) {
    int J[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) J[u] = bcol[s + u < re ? s + u : last];
    for (;;) {
      V kv[NB], zv[NB], pv[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int su = s + u < re ? s + u : last;
        kv[u] = load2<V>(K + 36 * (int64_t)su + off);
        zv[u] = load2<V>(z + 6 * (int64_t)J[u] + b);
        pv[u] = load2<V>(p + 6 * (int64_t)J[u] + b);
      }
      const int sn = s + NB;
      int Jn[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) Jn[u] = bcol[sn + u < re ? sn + u : last];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (s + u < re) {
          sz += kv[u].x * zv[u].x + kv[u].y * zv[u].y;
          sp += kv[u].x * pv[u].x + kv[u].y * pv[u].y;
        }
      s = sn;
      if (s >= re) break;
#pragma unroll
      for (int u = 0; u < NB; ++u) J[u] = Jn[u];
    }
  }
  az = sz;
  ap = sp;
}

// sum over the block row of K[s][a][b..b+1] . z and . p (two accumulators, so the products do
// not wait for beta): the direction's product is K p_new = Kz + beta Kp.  Two blocks per step.
// A step issues its K values and gathers together with the block columns of the next step, so
// a step costs one round trip to memory instead of two (the columns, then the gathers that
// need them); the products and their order are those of one block after another.
template <class T>
__device__ inline void row_product2(int rb, int re, const int32_t* __restrict__ bcol_,
                                    const T* __restrict__ K_, const T* __restrict__ z_,
                                    const T* __restrict__ p_, int a, int b, T& az, T& ap) {
  using V = typename Vec2<T>::type;
  const gptr<int32_t> bcol = as_global(bcol_);
  const gptr<T> K = as_global(K_);
  const gptr<T> z = as_global(z_);
  const gptr<T> p = as_global(p_);
  const int off = 6 * a + b;
  T sz = 0, sp = 0;
  int s = rb;
  if (re - rb >= 2) {
    int J0 = bcol[s], J1 = bcol[s + 1];
    for (;;) {
      const V k0 = load2<V>(K + 36 * (int64_t)s + off);
      const V k1 = load2<V>(K + 36 * (int64_t)(s + 1) + off);
      const V z0 = load2<V>(z + 6 * (int64_t)J0 + b);
      const V z1 = load2<V>(z + 6 * (int64_t)J1 + b);
      const V p0 = load2<V>(p + 6 * (int64_t)J0 + b);
      const V p1 = load2<V>(p + 6 * (int64_t)J1 + b);
      // the next step's columns; past the last pair, the row's last two (the odd block's
      // column is then the second)
      const int sn = s + 2;
      const int sc = sn + 2 <= re ? sn : re - 2;
      const int J0n = bcol[sc], J1n = bcol[sc + 1];
      sz += k0.x * z0.x + k0.y * z0.y;
      sp += k0.x * p0.x + k0.y * p0.y;
      sz += k1.x * z1.x + k1.y * z1.y;
      sp += k1.x * p1.x + k1.y * p1.y;
      s = sn;
      if (s + 2 > re) {
        if (s < re) {   // one block left: column bcol[re - 1] = J1n
          const V kv = load2<V>(K + 36 * (int64_t)s + off);
          const V zv = load2<V>(z + 6 * (int64_t)J1n + b);
          const V pv = load2<V>(p + 6 * (int64_t)J1n + b);
          sz += kv.x * zv.x + kv.y * zv.y;
          sp += kv.x * pv.x + kv.y * pv.y;
        }
        break;
      }
      J0 = J0n;
      J1 = J1n;
    }
  } else if (s < re) {
    const int J = bcol[s];
    const V kv = load2<V>(K + 36 * (int64_t)s + off);
    const V zv = load2<V>(z + 6 * (int64_t)J + b);
    const V pv = load2<V>(p + 6 * (int64_t)J + b);
    sz += kv.x * zv.x + kv.y * zv.y;
    sp += kv.x * pv.x + kv.y * pv.y;
  }
  az = sz;
  ap = sp;
}

// row_product2 reading only K's upper triangle (K is assembled bitwise symmetric): block s of
// row I with column J < I equals the transpose of block (J, I), so its entries (a, b) and
// (a, b + 1) are that block's (b, a) and (b + 1, a).  Each slot's (column, value slot) pair
// comes in one 8-byte load; the value slot is below s exactly for these blocks.  The values,
// the products and their order are row_product2's, so the sums are bitwise the same.  The
// mirrors are upper blocks of rows up to a grid line earlier, which the same XCD reads for
// those rows' own products at about the same time (xcd_tile): on the 300 x 300 shell the L2s
// fetch 172 MB per launch against 249 MB for the full K.  An upper block is one 16-byte load
// per lane, a mirror two 8-byte loads (stride 6); the choice is a branch per block, uniform
// within a wave away from the mesh's edges.  Measured per iteration on the 300 x 300 shell
// against 65.8 us for the full K: 57.1 us; two 8-byte loads for every block without the branch
// 62.0; a 16- and an 8-byte load 61.0-61.9; a scheduling barrier between a step's loads and its
// products 61.1; a register budget of 6 waves per SIMD 68.7.
template <class T>
__device__ inline void row_product2_sym(int rb, int re, const int32_t* __restrict__ bsym_,
                                        const T* __restrict__ K_, const T* __restrict__ z_,
                                        const T* __restrict__ p_, int a, int b, T& az, T& ap) {
  using V = typename Vec2<T>::type;
  const gptr<int32_t> bsym = as_global(bsym_);
  const gptr<T> K = as_global(K_);
  const gptr<T> z = as_global(z_);
  const gptr<T> p = as_global(p_);
  const int off_u = 6 * a + b, off_l = 6 * b + a;
  auto slot = [&](int s) { return load2<int2>(bsym + 2 * (int64_t)s); };   // (J, value slot)
  auto kval = [&](int s, int m) {
    V v;
    if (m < s) {
      const gptr<T> q = K + 36 * (int64_t)m + off_l;
      v.x = q[0];
      v.y = q[6];
    } else {
      v = load2<V>(K + 36 * (int64_t)m + off_u);
    }
    return v;
  };
  T sz = 0, sp = 0;
  int s = rb;
  if (re - rb >= 2) {
    int2 c0 = slot(s), c1 = slot(s + 1);
    for (;;) {
      // the next step's pairs (past the last pair, the row's last two), then this step's values
      // and gathers
      const int sn = s + 2;
      const int sc = sn + 2 <= re ? sn : re - 2;
      const int2 c0n = slot(sc), c1n = slot(sc + 1);
      const V k0 = kval(s, c0.y);
      const V k1 = kval(s + 1, c1.y);
      const V z0 = load2<V>(z + 6 * (int64_t)c0.x + b);
      const V z1 = load2<V>(z + 6 * (int64_t)c1.x + b);
      const V p0 = load2<V>(p + 6 * (int64_t)c0.x + b);
      const V p1 = load2<V>(p + 6 * (int64_t)c1.x + b);
      sz += k0.x * z0.x + k0.y * z0.y;
      sp += k0.x * p0.x + k0.y * p0.y;
      sz += k1.x * z1.x + k1.y * z1.y;
      sp += k1.x * p1.x + k1.y * p1.y;
      s = sn;
      if (s + 2 > re) {
        if (s < re) {   // one block left, slot re - 1: its pair is c1n
          const V kv = kval(s, c1n.y);
          const V zv = load2<V>(z + 6 * (int64_t)c1n.x + b);
          const V pv = load2<V>(p + 6 * (int64_t)c1n.x + b);
          sz += kv.x * zv.x + kv.y * zv.y;
          sp += kv.x * pv.x + kv.y * pv.y;
        }
        break;
      }
      c0 = c0n;
      c1 = c1n;
    }
  } else if (s < re) {
    const int2 c = slot(s);
    const V kv = kval(s, c.y);
    const V zv = load2<V>(z + 6 * (int64_t)c.x + b);
    const V pv = load2<V>(p + 6 * (int64_t)c.x + b);
    sz += kv.x * zv.x + kv.y * zv.y;
    sp += kv.x * pv.x + kv.y * pv.y;
  }
  az = sz;
  ap = sp;
}

// The tile (group of ROWS_PER_WG block rows) that workgroup lb of ng covers in each pass, as an
// offset into the pass's ng tiles.  Workgroups are dealt to the 8 XCDs in turn (lb mod 8), so
// this gives each XCD a contiguous range of the pass's tiles: the rows whose upper blocks a
// row's lower blocks mirror (a grid line back) are then mostly read by the same XCD.  A
// bijection of [0, ng); the per-workgroup partial sums follow the tiles a workgroup covers, so
// every launch of a problem (alone or in a multi-problem table) sums in the same order.
__device__ __forceinline__ int xcd_tile(int lb, int ng) {
  const int x = lb & 7, q = ng >> 3, r = ng & 7;
  return x * q + (x < r ? x : r) + (lb >> 3);
}

// FP64 products read only K's upper triangle (k_spmv_dir_sym) for a single solve whose K takes at
// least this many bytes, and in a multi-problem launch whose problems' K take that many together
// (the same sums either way).  Measured per iteration, full K against upper triangle: 300 x 300
// shell (234 MB) 65.8 against 57.1 us; 120 x 120 shell (38 MB, resident in the 256 MB Infinity
// Cache, where the bytes saved buy nothing) 18.7 against 19.8 us.  Launches of 24 / 32 / 48
// 60 x 60 shells: 2.80 / 2.99 / 3.20 against 2.97 / 3.29 / 3.24 us per problem-iteration (the
// full-K side with three blocks a step), the served stream 120.0 against 117.3 solves/s.
constexpr double SYM_PRODUCT_MIN_K_BYTES = 128.0 * 1024 * 1024;

// the upper-triangle product exists for FP64 only
template <class T>
constexpr bool spmv_sym_ok() {
  return sizeof(T) == 8;
}

template <class T>
static bool sym_products(const Pattern& pat) {
  return pcg_sym_products(pat.n_blocks, sizeof(T) != 8);
}

// FP32 standard recurrences keep z and p interleaved: buffer k holds (z, p) pairs, (z_j,
// p_{j-1}) in buffer j & 1, so that one 16-byte gather per lane brings both vectors' entries of
// a block (two entries each), where separate arrays need two 8-byte gathers.
template <class T>
constexpr bool zp_pairs() {
  return sizeof(T) == 4;
}

// row_product2 on interleaved (z, p) pairs: the same products in the same order, with the same
// global-address loads and the next step's block columns issued with the current step's loads.
__device__ inline void row_product2_zp(int rb, int re, const int32_t* __restrict__ bcol_,
                                       const float* __restrict__ K_,
                                       const float* __restrict__ zp_, int a, int b, float& az,
                                       float& ap) {
  typedef float N4 __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) N4* G4;
  const gptr<int32_t> bcol = as_global(bcol_);
  const gptr<float> K = as_global(K_);
  const gptr<float> zp = as_global(zp_);
  const int off = 6 * a + b;
  float sz = 0, sp = 0;
  int s = rb;
  if (re - rb >= 2) {
    int J0 = bcol[s], J1 = bcol[s + 1];
    for (;;) {
      const float2 k0 = load2<float2>(K + 36 * (int64_t)s + off);
      const float2 k1 = load2<float2>(K + 36 * (int64_t)(s + 1) + off);
      const N4 v0 = *(G4)(zp + 2 * (6 * (int64_t)J0 + b));
      const N4 v1 = *(G4)(zp + 2 * (6 * (int64_t)J1 + b));
      const int sn = s + 2;
      const int sc = sn + 2 <= re ? sn : re - 2;
      const int J0n = bcol[sc], J1n = bcol[sc + 1];
      sz += k0.x * v0.x + k0.y * v0.z;
      sp += k0.x * v0.y + k0.y * v0.w;
      sz += k1.x * v1.x + k1.y * v1.z;
      sp += k1.x * v1.y + k1.y * v1.w;
      s = sn;
      if (s + 2 > re) {
        if (s < re) {   // one block left: column bcol[re - 1] = J1n
          const float2 kv = load2<float2>(K + 36 * (int64_t)s + off);
          const N4 v = *(G4)(zp + 2 * (6 * (int64_t)J1n + b));
          sz += kv.x * v.x + kv.y * v.z;
          sp += kv.x * v.y + kv.y * v.w;
        }
        break;
      }
      J0 = J0n;
      J1 = J1n;
    }
  } else if (s < re) {
    const int J = bcol[s];
    const float2 kv = load2<float2>(K + 36 * (int64_t)s + off);
    const N4 v = *(G4)(zp + 2 * (6 * (int64_t)J + b));
    sz += kv.x * v.x + kv.y * v.z;
    sp += kv.x * v.y + kv.y * v.w;
  }
  az = sz;
  ap = sp;
}


// x = 0, r = b, z = Dinv b, p_{-1} = 0; partials of r^T z, r^T r; reset the state record.
template <class T>
__global__ void __launch_bounds__(MAX_TPB)
k_pcg_init(const PcgDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob, double rtol,
           int max_it) {
  __shared__ T rs[MAX_TPB];
  __shared__ __align__(16) T dl[DINV_PACKED * DINV_GROUP];
  const Wg<T> W = wg_of(D, wg_prob);
  const PcgDesc<T>& d = *W.d;
  const int n_nodes = d.n_nodes;
  T v[2] = {0, 0};
  for (int gi = W.lb; gi * VEC_NODES < n_nodes; gi += W.ng) {
    RowMap m = row_map_at(gi, n_nodes);
    const int64_t q = 6 * (int64_t)m.I + m.a;
    const DinvChunk<T> dc = dinv_load(d.Dinv, gi);
    T rv = 0;
    if (m.valid) {
      rv = d.b[q];
      d.x[q] = 0;
      d.r[q] = rv;
      if constexpr (!zp_pairs<T>()) d.p[0][q] = 0;
    }
    rs[threadIdx.x] = rv;
    dinv_stage(dc, dl);
    __syncthreads();
    if (m.valid) {
      const T zz = apply_dinv(dl, rs, m.a, m.lr);
      if constexpr (zp_pairs<T>()) {
        d.p[0][2 * q] = zz;
        d.p[0][2 * q + 1] = 0;
      } else {
        d.z[q] = zz;
      }
      v[0] += rv * zz;
      v[1] += rv * rv;
    }
    __syncthreads();
  }
  block_sum<2, T>(v);
  write_partials<2, T>(v, d.pb, W.lb, W.ng);
  if (W.lb == 0 && threadIdx.x == 0) {
    PcgState* st = d.st;
    st->rtol2 = rtol * rtol;
    st->max_it = max_it;
    st->it = 0;
    st->jn = 0;
    st->jc = 0;
    st->done = 0;
    st->status = SSO_OK;
  }
}

// The state scalars of a standard iteration, read at entry in one group: a kernel's later
// loads of the state would each be a round trip of their own after the done test.
struct StdState {
  double rz0, rz1, ff, rtol2;
  int done, jn, jc, max_it;
};

// A value every lane holds the same of, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)b);
  const long long hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The state is read through vector loads (other workgroups of the kernel write it, so scalar
// cache loads are not allowed); its fields are the same for every lane, so they are kept in
// scalar registers, where they cost no vector registers across the row products.
__device__ __forceinline__ StdState std_state(const PcgState* __restrict__ st) {
  StdState s;
  s.rz0 = uniform(st->rzs[0]);
  s.rz1 = uniform(st->rzs[1]);
  s.ff = uniform(st->ff);
  s.rtol2 = uniform(st->rtol2);
  s.max_it = __builtin_amdgcn_readfirstlane(st->max_it);
  s.done = __builtin_amdgcn_readfirstlane(st->done);
  s.jn = __builtin_amdgcn_readfirstlane(st->jn);
  s.jc = __builtin_amdgcn_readfirstlane(st->jc);
  return s;
}

// Iteration j (j read from the state), first half: Ap_j = K z_j + beta_j K p_{j-1} and
// p_j = z_j + beta_j p_{j-1} (own rows stored), partial p_j^T A p_j.  The first pass's products
// are issued before the previous kernel's partials are finished (rz_j, rr_j -> convergence
// test, beta_j), so the reduction overlaps the loads.  The descriptor is copied whole and the
// first pass's row pointers are loaded with the state (neither needs the other), so a
// workgroup's first products start two round trips after its descriptor.  SYM: the products
// read K's upper triangle only (row_product2_sym; bitwise the same sums).  EARLY: the update
// kernel's partials are issued with the state instead of after the first pass's products, so
// that finishing them costs no round trip of its own; the sums are the same.  Measured on the
// 300 x 300 shell (upper triangle, single solve): 54.3 against 55.4 us per iteration; in
// multi-problem launches, whose workgroups make one or two passes and lose a wave per SIMD to
// the registers on the two-block form, 2 % slower (the stream 0.8 %).
template <class T, int NB, bool SYM, bool EARLY, bool LEAD = false>
__device__ __forceinline__ void spmv_dir(const PcgDesc<T>* __restrict__ D,
                                         const int32_t* __restrict__ wg_prob,
                                         const int32_t* brow_ptr_l = nullptr,
                                         PcgState* st_l = nullptr, const double* pb_l = nullptr,
                                         int n_nodes_l = 0, int n_wg_l = 0) {
  static_assert(!SYM || (NB == 2 && !zp_pairs<T>()), "symmetric products: FP64, two blocks a step");
  PcgDesc<T> d = D[wg_prob ? wg_prob[blockIdx.x] : 0];
  if constexpr (LEAD) {   // single problem: the first group's fields from preloaded arguments
    d.brow_ptr = brow_ptr_l;
    d.st = st_l;
    d.pb = const_cast<double*>(pb_l);
    d.n_nodes = n_nodes_l;
    d.n_wg = n_wg_l;
    d.wg_base = 0;
  }
  const int lb = (int)blockIdx.x - d.wg_base, ng = d.n_wg;
  PcgState* st = d.st;
  const int n_nodes = d.n_nodes;
  const SpLane L = sp_lane();
  const int wave = threadIdx.x >> 6;
  const int t0 = xcd_tile(lb, ng);
  const int I0 = t0 * ROWS_PER_WG + wave * ROWS_PER_WAVE + L.g;
  const int I0c = (L.ok && I0 < n_nodes) ? I0 : 0;
  const int rb0 = d.brow_ptr[I0c], re0 = d.brow_ptr[I0c + 1];
  // EARLY: the update kernel's partials of r^T z and r^T r, issued with the state (at most
  // three per thread and sum), summed after the first pass's products in finish_partials' order
  double pb6[2][3] = {};
  if constexpr (EARLY) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int k = (int)threadIdx.x + u * MAX_TPB;
        pb6[c][u] = d.pb[c * ng + (k < ng ? k : 0)];
      }
  }
  const StdState S = std_state(st);
  // the first group in registers before the done test (an empty asm that takes them), so that
  // the compiler cannot sink these loads below it, one round trip after another
  asm volatile("" ::"v"(rb0), "v"(re0), "s"(S.rz0), "s"(S.rz1), "s"(S.ff), "s"(S.rtol2),
               "s"(S.jn), "s"(S.max_it));
  if (S.done) return;
  const int j = S.jn;
  const T* __restrict__ K = d.K;
  const T* __restrict__ z = d.z;
  const T* __restrict__ pold = (j & 1) ? d.p[1] : d.p[0];
  T* __restrict__ pnew = (j & 1) ? d.p[0] : d.p[1];
  T* __restrict__ Ap = d.Ap;
  T beta = 0, my = 0;
  // (issuing the next pass's row pointers during a pass measured slower: 56.3 against 55.9 us
  // per iteration on the 300 x 300 shell, 1-2 % on multi-problem launches)
  for (int gi = t0; gi * ROWS_PER_WG < n_nodes; gi += ng) {
    const int I = gi * ROWS_PER_WG + wave * ROWS_PER_WAVE + L.g;
    const bool ok = L.ok && I < n_nodes;
    T az = 0, ap = 0, zI = 0, pI = 0;
    int rb = rb0, re = re0;
    if (gi != t0 && ok) {
      rb = d.brow_ptr[I];
      re = d.brow_ptr[I + 1];
    }
    if (!ok) re = rb;
    if constexpr (zp_pairs<T>()) {
      row_product2_zp(rb, re, d.bcol, K, pold, L.a, L.b, az, ap);
      if (ok && L.b == 0) {
        zI = pold[2 * (6 * (int64_t)I + L.a)];
        pI = pold[2 * (6 * (int64_t)I + L.a) + 1];
      }
    } else {
      if constexpr (SYM)
        row_product2_sym<T>(rb, re, d.bsym, K, z, pold, L.a, L.b, az, ap);
      else if constexpr (NB == 2)
        row_product2<T>(rb, re, d.bcol, K, z, pold, L.a, L.b, az, ap);
      else
        row_product_nb<T, NB>(rb, re, d.bcol, K, z, pold, L.a, L.b, az, ap);
      if (ok && L.b == 0) {
        zI = z[6 * (int64_t)I + L.a];
        pI = pold[6 * (int64_t)I + L.a];
      }
    }
    if (gi == t0) {
      double tot[2];
      if constexpr (EARLY) {
        const int k0 = (int)threadIdx.x;
#pragma unroll
        for (int c = 0; c < 2; ++c)
          tot[c] = ((0.0 + (k0 < ng ? pb6[c][0] : 0.0)) + (k0 + MAX_TPB < ng ? pb6[c][1] : 0.0)) +
                   (k0 + 2 * MAX_TPB < ng ? pb6[c][2] : 0.0);
        block_sum<2, double>(tot);
      } else {
        finish_partials<2>(d.pb, ng, tot);
      }
      const double rz = tot[0], rr = tot[1];
      const double ff = (j == 0) ? rr : S.ff;
      const double beta_d = (j == 0) ? 0.0 : rz / ((j & 1) ? S.rz0 : S.rz1);
      int stop = 0, status = SSO_OK;
      if (!std::isfinite(rr) || !std::isfinite(rz)) {
        stop = 1;
        status = SSO_EBREAKDOWN;
      } else if (rr <= S.rtol2 * ff) {
        stop = 1;
      } else if (j >= S.max_it) {
        stop = 1;
        status = SSO_ENOTCONV;
      }
      if (lb == 0 && threadIdx.x == 0) {
        st->rzs[j & 1] = rz;
        st->rr = rr;
        st->it = j;
        st->jc = j;
        if (j == 0) st->ff = rr;
        if (stop) {
          st->status = status;
          st->done = 1;
        }
      }
      if (stop) return;
      beta = (T)beta_d;
    }
    const T sz = sum3(az), sp = sum3(ap);
    if (ok && L.b == 0) {
      const int64_t q = 6 * (int64_t)I + L.a;
      const T pn = zI + beta * pI;
      const T Apq = sz + beta * sp;
      if constexpr (zp_pairs<T>())
        put(&pnew[2 * q + 1], pn, d.stream_stores);
      else
        put(&pnew[q], pn, d.stream_stores);
      put(&Ap[q], Apq, d.stream_stores);
      my += pn * Apq;
    }
  }
  T v[1] = {my};
  block_sum<1, T>(v);
  write_partials<1, T>(v, d.pa, lb, ng);
}

template <class T, int NB = 2>
__global__ void __launch_bounds__(MAX_TPB)
k_spmv_dir(const PcgDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  spmv_dir<T, NB, false, false>(D, wg_prob);
}

// The upper-triangle form for multi-problem launches (66 VGPRs, 7 waves per SIMD; single solves
// take k_spmv_dir_single, 70 with its early partials).  A
// three-blocks-per-step form for multi-problem launches of more than 1,024 workgroups (80 VGPRs,
// 6 waves) measured 3.0-3.4 against 2.78-3.13 us per problem-iteration on 24-48 60 x 60 shells
// and the served stream 114.6-115.0 against 122.9-123.2 solves/s, and was not kept.
template <class T>
__global__ void __launch_bounds__(MAX_TPB)
k_spmv_dir_sym(const PcgDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  spmv_dir<T, 2, true, false>(D, wg_prob);
}

// Single problems: the fields of the first group of loads (row pointers, state, the update
// kernel's partials, sizes) as leading scalar arguments, which arrive preloaded in SGPRs, so
// those loads do not wait for the descriptor; the descriptor brings the rest meanwhile.  SYM:
// the upper-triangle products, with the partials issued with the state (EARLY).
template <class T, bool SYM>
__global__ void __launch_bounds__(MAX_TPB)
k_spmv_dir_single(const int32_t* brow_ptr, PcgState* st, const double* pb, int n_nodes, int n_wg,
                  const PcgDesc<T>* __restrict__ D) {
  spmv_dir<T, 2, SYM, SYM, true>(D, nullptr, brow_ptr, st, pb, n_nodes, n_wg);
}

// Iteration j, second half: finish pAp_j, alpha_j; x += alpha p, r -= alpha Ap, z = Dinv r,
// partials of (rz_{j+1}, rr_{j+1}); the state's next iteration index becomes j + 1.  The first
// pass's operands (x, Ap, r, p of both parities, the inverses) and the product kernel's partials
// are loaded with the state itself, so the reduction and the updates wait for one round trip.
// LEAD (single problems): the sizes, Ap, r, both p buffers, the product kernel's partials and
// the state come as preloaded arguments (14 dwords, as many as are preloaded), so the first
// group of loads goes out at once; x and the inverses, not needed before alpha, come with the
// descriptor, their loads issued after the others'.
template <class T, bool LEAD>
__device__ __forceinline__ void update_body(const PcgDesc<T>* __restrict__ D,
                                            const int32_t* __restrict__ wg_prob, int n_nodes_l,
                                            int n_wg_l, const T* Ap_l, T* r_l, T* p0_l,
                                            T* p1_l, const double* pa_l, PcgState* st_l) {
  __shared__ T rs[MAX_TPB];
  __shared__ __align__(16) T dl[DINV_PACKED * DINV_GROUP];
  PcgDesc<T> d = D[wg_prob ? wg_prob[blockIdx.x] : 0];
  if constexpr (LEAD) {
    d.Ap = const_cast<T*>(Ap_l);
    d.r = r_l;
    d.p[0] = p0_l;
    d.p[1] = p1_l;
    d.pa = const_cast<double*>(pa_l);
    d.st = st_l;
    d.n_nodes = n_nodes_l;
    d.n_wg = n_wg_l;
    d.wg_base = 0;
  } else {
    // every field the kernel uses in one batch of scalar loads
    asm volatile("" ::"s"(d.x), "s"(d.r), "s"(d.z), "s"(d.p[0]), "s"(d.p[1]), "s"(d.Ap),
                 "s"(d.Dinv), "s"(d.pa), "s"(d.pb), "s"(d.st), "s"(d.n_nodes), "s"(d.n_wg),
                 "s"(d.wg_base), "s"(d.stream_stores));
  }
  const int lb = (int)blockIdx.x - d.wg_base, ng = d.n_wg;
  PcgState* st = d.st;
  const int n_nodes = d.n_nodes;
  T* __restrict__ x = d.x;
  T* __restrict__ r = d.r;
  T* __restrict__ z = d.z;
  const T* __restrict__ Ap = d.Ap;
  const RowMap m0 = row_map_at(lb, n_nodes);
  const int64_t q0 = 6 * (int64_t)(m0.valid ? m0.I : 0) + m0.a;
  T x0 = 0;
  if constexpr (!LEAD) x0 = x[q0];
  const T a0 = Ap[q0], r0 = r[q0];
  // the first pass's inverses, state-free; a workgroup with no node group of its own (the
  // launch has one workgroup per 18 block rows, a group is 64 nodes) reads group 0 and drops it
  // (LEAD: issued after the preloaded group, below)
  DinvChunk<T> dc0{};
  if constexpr (!LEAD) dc0 = dinv_load(d.Dinv, lb * VEC_NODES < n_nodes ? lb : 0);
  // Issued with the state, which neither needs: the product kernel's partials of p^T A p (at
  // most three per thread: ng <= PCG_MAX_WG <= 3 MAX_TPB), summed below in finish_partials'
  // order, and the first pass's p from both parity buffers (the state names which is p_j).
  // Waiting for the state first and then for these cost a second round trip: on the 300 x 300
  // shell 55.8 against 56.6 us per iteration (two alternating runs each).
  static_assert(3 * MAX_TPB >= PCG_MAX_WG, "three partials per thread");
  double pa3[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int k = (int)threadIdx.x + u * MAX_TPB;
    pa3[u] = d.pa[k < ng ? k : 0];
  }
  const int64_t qp0 = zp_pairs<T>() ? 2 * q0 + 1 : q0;
  const T p0e = d.p[0][qp0], p1e = d.p[1][qp0];
  const StdState S = std_state(st);
  if constexpr (LEAD) {
    x0 = x[q0];
    dc0 = dinv_load(d.Dinv, lb * VEC_NODES < n_nodes ? lb : 0);
  }
  asm volatile("" ::"v"(x0), "v"(a0), "v"(r0), "s"(S.rz0), "s"(S.rz1), "s"(S.jc));
  if (S.done) return;
  const int j = S.jc;
  T* __restrict__ p = (j & 1) ? d.p[0] : d.p[1];   // p_j (FP32: beside z_{j+1}, written here)
  T alpha = 0;
  T v[2] = {0, 0};
  for (int gi = lb; gi * VEC_NODES < n_nodes; gi += ng) {
    RowMap m = row_map_at(gi, n_nodes);
    const int64_t q = 6 * (int64_t)m.I + m.a;
    T xv = x0, pv = 0, av = a0, rv = r0;
    if (m.valid) {
      if (gi != lb) {
        xv = x[q];
        av = Ap[q];
        rv = r[q];
        pv = zp_pairs<T>() ? p[2 * q + 1] : p[q];
      } else {
        pv = (j & 1) ? p0e : p1e;
      }
    }
    if (gi == lb) {
      double tot[1];
      {
        const int k0 = (int)threadIdx.x;
        tot[0] = ((0.0 + (k0 < ng ? pa3[0] : 0.0)) + (k0 + MAX_TPB < ng ? pa3[1] : 0.0)) +
                 (k0 + 2 * MAX_TPB < ng ? pa3[2] : 0.0);
        block_sum<1, double>(tot);
      }
      const double pAp = tot[0];
      const double alpha_d = ((j & 1) ? S.rz1 : S.rz0) / pAp;
      if (!(pAp > 0.0) || !std::isfinite(alpha_d)) {
        if (lb == 0 && threadIdx.x == 0) {
          st->status = SSO_EBREAKDOWN;
          st->done = 1;
        }
        return;
      }
      alpha = (T)alpha_d;
    }
    T rn = 0;
    if (m.valid) {
      put(&x[q], xv + alpha * pv, d.stream_stores);
      rn = rv - alpha * av;
      put(&r[q], rn, d.stream_stores);
    }
    rs[threadIdx.x] = rn;
    dinv_stage(gi == lb ? dc0 : dinv_load(d.Dinv, gi), dl);
    __syncthreads();
    if (m.valid) {
      const T zz = apply_dinv(dl, rs, m.a, m.lr);
      if constexpr (zp_pairs<T>())
        put(&p[2 * q], zz, d.stream_stores);   // z_{j+1} beside p_j
      else
        put(&z[q], zz, d.stream_stores);
      v[0] += rn * zz;
      v[1] += rn * rn;
    }
    __syncthreads();
  }
  block_sum<2, T>(v);
  write_partials<2, T>(v, d.pb, lb, ng);
  if (lb == 0 && threadIdx.x == 0) st->jn = j + 1;
}

template <class T>
__global__ void __launch_bounds__(MAX_TPB)
k_update(const PcgDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  update_body<T, false>(D, wg_prob, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

template <class T>
__global__ void __launch_bounds__(MAX_TPB)
k_update_single(int n_nodes, int n_wg, const T* Ap, T* r, T* p0, T* p1, const double* pa,
                PcgState* st, const PcgDesc<T>* __restrict__ D) {
  update_body<T, true>(D, nullptr, n_nodes, n_wg, Ap, r, p0, p1, pa, st);
}

// ---- one workgroup per problem: every iteration inside one launch ----------------------------
// For the smallest problems an iteration of the kernel pair is a few microseconds of launch and
// round-trip latency around almost no data.  Here one workgroup of 16 waves holds a whole
// problem and runs the standard recurrences with workgroup barriers between the phases (no grid
// synchronisation); several problems share a launch, one workgroup each.  The block-row products
// are the pair's (row_product2), so only the order of the three reductions differs.  Between
// launches the state record carries rz_j, rz_{j-1} and rr_j, so a launch resumes where the last
// one stopped.
constexpr int WG1_TPB = 1024;
constexpr int WG1_WAVES = WG1_TPB / 64;
constexpr int WG1_ROWS = ROWS_PER_WAVE * WG1_WAVES;   // 48 block rows per product pass
constexpr int WG1_NODE_LANES = 60;                    // 10 nodes a wave in the vector pass
constexpr int WG1_NODES = (WG1_NODE_LANES / 6) * WG1_WAVES;   // 160 nodes per vector pass

// Fixed-order sum of NV values over the 16 waves, returned to every thread; ends with a barrier
// (the LDS array is reused by the next call, and the phase that follows reads what other waves
// wrote before the call).
template <int NV>
__device__ inline void wg1_sum(double v[NV]) {
  __shared__ double lds[NV][WG1_WAVES];
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < NV; ++k) lds[k][wave] = v[k];
  __syncthreads();
  for (int k = 0; k < NV; ++k) {
    double t = lds[k][0];
    for (int w = 1; w < WG1_WAVES; ++w) t += lds[k][w];
    v[k] = t;
  }
  __syncthreads();
}

// Up to n_iter iterations of one problem, its vectors in global memory (descriptor d; its n_wg,
// wg_base, pa and pb are not used).  At j = 0 (x = 0, r = b, z = Dinv b, p_{-1} = 0 from the
// initialisation kernel) it forms r^T z and r^T r itself.  The stopping test is the standard
// pair's, on r_j^T r_j against rtol^2 |b|^2.
__device__ inline void wg_global(const PcgDesc<double>& d, int n_iter) {
  PcgState* st = d.st;
  const int n = d.n_nodes;
  const StdState S = std_state(st);
  if (S.done) return;
  const SpLane L = sp_lane();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n_dof = 6 * (int64_t)n;
  int j = S.jn;
  double rz, rzp = 1.0, rr, ff = S.ff;
  if (j == 0) {
    double v[2] = {0.0, 0.0};
    for (int64_t q = threadIdx.x; q < n_dof; q += WG1_TPB) {
      const double rq = d.r[q];
      v[0] += rq * d.z[q];
      v[1] += rq * rq;
    }
    wg1_sum<2>(v);
    rz = v[0];
    rr = v[1];
    ff = rr;
  } else {
    rz = (j & 1) ? S.rz1 : S.rz0;
    rzp = (j & 1) ? S.rz0 : S.rz1;
    rr = uniform(st->rr);
  }
  const int j_end = j + n_iter;
  int stop = 0, status = SSO_OK;
  for (;; ++j) {
    if (!std::isfinite(rr) || !std::isfinite(rz)) {
      stop = 1;
      status = SSO_EBREAKDOWN;
    } else if (rr <= S.rtol2 * ff) {
      stop = 1;
    } else if (j >= S.max_it) {
      stop = 1;
      status = SSO_ENOTCONV;
    }
    if (stop || j >= j_end) break;
    const double beta = (j == 0) ? 0.0 : rz / rzp;
    const double* __restrict__ pold = (j & 1) ? d.p[1] : d.p[0];
    double* __restrict__ pnew = (j & 1) ? d.p[0] : d.p[1];
    // Ap_j = K z_j + beta K p_{j-1}, p_j = z_j + beta p_{j-1}; partial p_j^T Ap_j
    double my = 0.0;
    for (int I0 = 0; I0 < n; I0 += WG1_ROWS) {
      const int I = I0 + wave * ROWS_PER_WAVE + L.g;
      const bool ok = L.ok && I < n;
      int rb = 0, re = 0;
      if (ok) {
        rb = d.brow_ptr[I];
        re = d.brow_ptr[I + 1];
      }
      double az, ap;
      row_product2<double>(rb, re, d.bcol, d.K, d.z, pold, L.a, L.b, az, ap);
      const double sz = sum3(az), sp = sum3(ap);
      if (ok && L.b == 0) {
        const int64_t q = 6 * (int64_t)I + L.a;
        const double pn = d.z[q] + beta * pold[q];
        const double Apq = sz + beta * sp;
        pnew[q] = pn;
        d.Ap[q] = Apq;
        my += pn * Apq;
      }
    }
    double pap[1] = {my};
    wg1_sum<1>(pap);
    const double alpha = rz / pap[0];
    // x += alpha p_j, r -= alpha Ap_j, z = Dinv r (a node's six r values by wave shuffles);
    // partials of r^T z and r^T r
    double v[2] = {0.0, 0.0};
    const int k = lane / 6, a = lane - 6 * k;
    for (int I0 = 0; I0 < n; I0 += WG1_NODES) {
      const int I = I0 + wave * (WG1_NODE_LANES / 6) + k;
      const bool ok = lane < WG1_NODE_LANES && I < n;
      const int64_t q = 6 * (int64_t)I + a;
      double rv = 0.0;
      if (ok) {
        d.x[q] += alpha * pnew[q];
        rv = d.r[q] - alpha * d.Ap[q];
        d.r[q] = rv;
      }
      double rn[6];
      for (int c = 0; c < 6; ++c) rn[c] = __shfl(rv, 6 * k + c, 64);
      if (ok) {
        const double zq = dinv_row(d.Dinv, I, a).apply(rn);
        d.z[q] = zq;
        v[0] += rv * zq;
        v[1] += rv * rv;
      }
    }
    wg1_sum<2>(v);
    rzp = rz;
    rz = v[0];
    rr = v[1];
  }
  if (threadIdx.x == 0) {
    st->rzs[j & 1] = rz;
    st->rzs[(j + 1) & 1] = rzp;
    st->rr = rr;
    st->ff = ff;
    st->it = j;
    st->jc = j;
    st->jn = j;
    if (stop) {
      st->status = status;
      st->done = 1;
    }
  }
}

// The same iterations with the problem resident in the workgroup's LDS, for problems of at most
// WGL_MAX_NODES nodes whose gathered vectors and pattern fit it (wgl_bytes): z, p_{j-1} and p_j,
// the block columns and the row pointers are staged once per launch.  Each lane that owns a DOF
// (the first of its 3-lane set, as in the products) keeps the DOF's x and r in registers for the
// whole launch and uses the same mapping in both phases; Ap and p_j pass between the phases
// through LDS, a node's six r values come by wave shuffles, and the packed inverses are staged
// in LDS too.  Only K is read from memory each iteration.  The products, and their order, are those of the global path; the
// reduction trees differ (lanes, not 60-lane node groups, in the second phase).
constexpr int WGL_PASSES = 3;
constexpr int WGL_MAX_NODES = WG1_ROWS * WGL_PASSES;   // 144
constexpr int WGL_LDS_BYTES = 60 * 1024;
__host__ __device__ inline int64_t wgl_bytes(int64_t n_nodes, int64_t n_blocks) {
  return (4 * 6 + DINV_PACKED) * 8 * n_nodes + 4 * (n_nodes + 1 + n_blocks);
}

// row_product2 with the block columns and the gathered vectors in LDS (K from memory), three
// blocks a step so that a step's K loads are in flight together.
__device__ inline void row_product_lds(int rb, int re, const int32_t* bcl,
                                       const double* __restrict__ K_, const double* zl,
                                       const double* pl, int a, int b, double& az,
                                       double& ap) {
  const gptr<double> K = as_global(K_);
  const int off = 6 * a + b;
  double sz = 0, sp = 0;
  int s = rb;
  for (; s + 3 <= re; s += 3) {
    const int J0 = bcl[s], J1 = bcl[s + 1], J2 = bcl[s + 2];
    const double2 k0 = load2<double2>(K + 36 * (int64_t)s + off);
    const double2 k1 = load2<double2>(K + 36 * (int64_t)(s + 1) + off);
    const double2 k2 = load2<double2>(K + 36 * (int64_t)(s + 2) + off);
    const double2 z0 = *reinterpret_cast<const double2*>(zl + 6 * J0 + b);
    const double2 z1 = *reinterpret_cast<const double2*>(zl + 6 * J1 + b);
    const double2 z2 = *reinterpret_cast<const double2*>(zl + 6 * J2 + b);
    const double2 p0 = *reinterpret_cast<const double2*>(pl + 6 * J0 + b);
    const double2 p1 = *reinterpret_cast<const double2*>(pl + 6 * J1 + b);
    const double2 p2 = *reinterpret_cast<const double2*>(pl + 6 * J2 + b);
    sz += k0.x * z0.x + k0.y * z0.y;
    sp += k0.x * p0.x + k0.y * p0.y;
    sz += k1.x * z1.x + k1.y * z1.y;
    sp += k1.x * p1.x + k1.y * p1.y;
    sz += k2.x * z2.x + k2.y * z2.y;
    sp += k2.x * p2.x + k2.y * p2.y;
  }
  for (; s < re; ++s) {
    const int J = bcl[s];
    const double2 kv = load2<double2>(K + 36 * (int64_t)s + off);
    const double2 zv = *reinterpret_cast<const double2*>(zl + 6 * J + b);
    const double2 pv = *reinterpret_cast<const double2*>(pl + 6 * J + b);
    sz += kv.x * zv.x + kv.y * zv.y;
    sp += kv.x * pv.x + kv.y * pv.y;
  }
  az = sz;
  ap = sp;
}

__device__ inline void wg_lds(const PcgDesc<double>& d, int n_iter, unsigned char* smem) {
  PcgState* st = d.st;
  const int n = d.n_nodes;
  const int n6 = 6 * n;
  const StdState S = std_state(st);
  if (S.done) return;
  const SpLane L = sp_lane();
  const int wave = threadIdx.x >> 6;
  double* zl = reinterpret_cast<double*>(smem);
  double* pl0 = zl + n6;
  double* pl1 = pl0 + n6;
  double* apl = pl1 + n6;
  double* dl = apl + n6;   // packed inverses, DINV_PACKED per node
  int32_t* rpl = reinterpret_cast<int32_t*>(dl + DINV_PACKED * n);
  int32_t* bcl = rpl + (n + 1);
  const gptr<int32_t> brow = as_global(d.brow_ptr);
  int j = S.jn;
  {
    const int nbk = brow[n];
    const gptr<int32_t> bc = as_global(d.bcol);
    for (int i = threadIdx.x; i <= n; i += WG1_TPB) rpl[i] = brow[i];
    for (int i = threadIdx.x; i < nbk; i += WG1_TPB) bcl[i] = bc[i];
    const gptr<double> zg = as_global(d.z);
    const gptr<double> pg = as_global((j & 1) ? d.p[1] : d.p[0]);   // p_{j-1}
    double* po = (j & 1) ? pl1 : pl0;
    for (int q = threadIdx.x; q < n6; q += WG1_TPB) {
      zl[q] = zg[q];
      po[q] = pg[q];
    }
    const gptr<double> dg = as_global(d.Dinv);
    for (int i = threadIdx.x; i < DINV_PACKED * n; i += WG1_TPB) dl[i] = dg[i];
  }
  const bool owner = L.ok && L.b == 0;
  double xk[WGL_PASSES], rk[WGL_PASSES];
#pragma unroll
  for (int k = 0; k < WGL_PASSES; ++k) {
    const int I = k * WG1_ROWS + wave * ROWS_PER_WAVE + L.g;
    xk[k] = 0.0;
    rk[k] = 0.0;
    if (owner && I < n) {
      const int64_t q = 6 * (int64_t)I + L.a;
      xk[k] = as_global(d.x)[q];
      rk[k] = as_global(d.r)[q];
    }
  }
  __syncthreads();
  double rz, rzp = 1.0, rr, ff = S.ff;
  if (j == 0) {
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < WGL_PASSES; ++k) {
      const int I = k * WG1_ROWS + wave * ROWS_PER_WAVE + L.g;
      if (owner && I < n) {
        v[0] += rk[k] * zl[6 * I + L.a];
        v[1] += rk[k] * rk[k];
      }
    }
    wg1_sum<2>(v);
    rz = v[0];
    rr = v[1];
    ff = rr;
  } else {
    rz = (j & 1) ? S.rz1 : S.rz0;
    rzp = (j & 1) ? S.rz0 : S.rz1;
    rr = uniform(st->rr);
  }
  const int j_end = j + n_iter;
  int stop = 0, status = SSO_OK;
  for (;; ++j) {
    if (!std::isfinite(rr) || !std::isfinite(rz)) {
      stop = 1;
      status = SSO_EBREAKDOWN;
    } else if (rr <= S.rtol2 * ff) {
      stop = 1;
    } else if (j >= S.max_it) {
      stop = 1;
      status = SSO_ENOTCONV;
    }
    if (stop || j >= j_end) break;
    const double beta = (j == 0) ? 0.0 : rz / rzp;
    const double* po = (j & 1) ? pl1 : pl0;   // p_{j-1}
    double* pnl = (j & 1) ? pl0 : pl1;        // p_j
    double my = 0.0;
#pragma unroll 1
    for (int k = 0; k * WG1_ROWS < n; ++k) {
      const int I = k * WG1_ROWS + wave * ROWS_PER_WAVE + L.g;
      const bool ok = L.ok && I < n;
      int rb = 0, re = 0;
      if (ok) {
        rb = rpl[I];
        re = rpl[I + 1];
      }
      double az, ap;
      row_product_lds(rb, re, bcl, d.K, zl, po, L.a, L.b, az, ap);
      const double sz = sum3(az), sp = sum3(ap);
      if (ok && L.b == 0) {
        const int q = 6 * I + L.a;
        const double pn = zl[q] + beta * po[q];
        const double Apq = sz + beta * sp;
        pnl[q] = pn;
        apl[q] = Apq;
        my += pn * Apq;
      }
    }
    double pap[1] = {my};
    wg1_sum<1>(pap);
    const double alpha = rz / pap[0];
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < WGL_PASSES; ++k) {
      if (k * WG1_ROWS >= n) continue;
      const int I = k * WG1_ROWS + wave * ROWS_PER_WAVE + L.g;
      const bool ok = owner && I < n;
      if (ok) {
        const int q = 6 * I + L.a;   // written by this lane in the product phase
        xk[k] += alpha * pnl[q];
        rk[k] -= alpha * apl[q];
      }
      double rn[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) rn[c] = __shfl(rk[k], ROW_LANES * L.g + 3 * c, 64);
      if (ok) {
        const double* dn = dl + DINV_PACKED * I;
        double zq = 0;
#pragma unroll
        for (int h = 0; h < 3; ++h)
          zq += dn[dinv_index(L.a, 2 * h)] * rn[2 * h] +
                dn[dinv_index(L.a, 2 * h + 1)] * rn[2 * h + 1];
        zl[6 * I + L.a] = zq;
        v[0] += rk[k] * zq;
        v[1] += rk[k] * rk[k];
      }
    }
    wg1_sum<2>(v);
    rzp = rz;
    rz = v[0];
    rr = v[1];
  }
  // back to memory: x and r of the owned DOFs, z and p_{j-1} of the next launch
#pragma unroll
  for (int k = 0; k < WGL_PASSES; ++k) {
    const int I = k * WG1_ROWS + wave * ROWS_PER_WAVE + L.g;
    if (owner && I < n) {
      const int64_t q = 6 * (int64_t)I + L.a;
      d.x[q] = xk[k];
      d.r[q] = rk[k];
    }
  }
  {
    double* pg = (j & 1) ? d.p[1] : d.p[0];
    const double* po = (j & 1) ? pl1 : pl0;
    for (int q = threadIdx.x; q < n6; q += WG1_TPB) {
      d.z[q] = zl[q];
      pg[q] = po[q];
    }
  }
  if (threadIdx.x == 0) {
    st->rzs[j & 1] = rz;
    st->rzs[(j + 1) & 1] = rzp;
    st->rr = rr;
    st->ff = ff;
    st->it = j;
    st->jc = j;
    st->jn = j;
    if (stop) {
      st->status = status;
      st->done = 1;
    }
  }
}

// One problem per workgroup (descriptor D[blockIdx.x]): resident in LDS when it fits the
// lds_bytes of dynamic LDS the launch provides, else from global memory.
__global__ void __launch_bounds__(WG1_TPB)
k_pcg_wg(const PcgDesc<double>* __restrict__ D, int n_iter, int lds_bytes) {
  extern __shared__ __align__(16) unsigned char wg_smem[];
  const PcgDesc<double> d = D[blockIdx.x];
  const int n = d.n_nodes;
  if (n <= WGL_MAX_NODES && wgl_bytes(n, as_global(d.brow_ptr)[n]) <= (int64_t)lds_bytes)
    wg_lds(d, n_iter, wg_smem);
  else
    wg_global(d, n_iter);
}

// ---- single-reduction PCG (Chronopoulos & Gear): one kernel and one reduction per iteration --
//
// The recurrences carry s = K p beside p, and w = K M r (M the block-Jacobi inverse) comes from
// an SpMV with B = K M, which has the block pattern of K because M is block diagonal.  With
// r_i, w_i, s_{i-1} stored and the partial sums of gamma_i = r_i.M r_i, delta_i = w_i.M r_i and
// rho_i = r_i.r_i left by the previous launch, iteration i is
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta_i - beta gamma_i / alpha_{i-1})
//   p_i = M r_i + beta p_{i-1};  s_i = w_i + beta s_{i-1};  x += alpha p_i;  r_{i+1} = r_i - alpha s_i
//   w_{i+1} = B r_{i+1} = B r_i - alpha B w_i - alpha beta B s_{i-1}
// and partials of gamma_{i+1}, delta_{i+1}, rho_{i+1}.  The three products of the last line use
// stored vectors only, so no workgroup waits for another inside a launch; their loads are issued
// before the previous partials are finished.  r, w, s and the partials are double-buffered by
// iteration parity and every workgroup keeps its own iteration counter.

// sum over the block slots [rb, re) of one block row of B[s][a][b..b+1] . (r, w, t) (three
// accumulators).
template <class T>
__device__ inline void row_product3(int rb, int re, const int32_t* __restrict__ bcol,
                                    const T* __restrict__ B, const T* __restrict__ r,
                                    const T* __restrict__ w, const T* __restrict__ t, int a,
                                    int b, T& ar, T& aw, T& at) {
  using V = typename Vec2<T>::type;
  const int off = 6 * a + b;
  T sr = 0, sw = 0, st = 0;
  int s = rb;
  for (; s + 2 <= re; s += 2) {
    const int64_t J0 = bcol[s], J1 = bcol[s + 1];
    const V k0 = *reinterpret_cast<const V*>(B + 36 * (int64_t)s + off);
    const V k1 = *reinterpret_cast<const V*>(B + 36 * (int64_t)(s + 1) + off);
    const V r0 = *reinterpret_cast<const V*>(r + 6 * J0 + b);
    const V r1 = *reinterpret_cast<const V*>(r + 6 * J1 + b);
    const V w0 = *reinterpret_cast<const V*>(w + 6 * J0 + b);
    const V w1 = *reinterpret_cast<const V*>(w + 6 * J1 + b);
    const V t0 = *reinterpret_cast<const V*>(t + 6 * J0 + b);
    const V t1 = *reinterpret_cast<const V*>(t + 6 * J1 + b);
    sr += k0.x * r0.x + k0.y * r0.y;
    sw += k0.x * w0.x + k0.y * w0.y;
    st += k0.x * t0.x + k0.y * t0.y;
    sr += k1.x * r1.x + k1.y * r1.y;
    sw += k1.x * w1.x + k1.y * w1.y;
    st += k1.x * t1.x + k1.y * t1.y;
  }
  if (s < re) {
    const int64_t J = bcol[s];
    const V kv = *reinterpret_cast<const V*>(B + 36 * (int64_t)s + off);
    const V rv = *reinterpret_cast<const V*>(r + 6 * J + b);
    const V wv = *reinterpret_cast<const V*>(w + 6 * J + b);
    const V tv = *reinterpret_cast<const V*>(t + 6 * J + b);
    sr += kv.x * rv.x + kv.y * rv.y;
    sw += kv.x * wv.x + kv.y * wv.y;
    st += kv.x * tv.x + kv.y * tv.y;
  }
  ar = sr;
  aw = sw;
  at = st;
}

// The same over the W padded slots of row I (B in the padded layout, bcol_ell): every load
// address is known without the row pointers, the padding adds exact zeros.
// The row's column indices and this lane's entries of its W blocks (addresses from the row
// index alone).
template <class T, int W>
struct EllRow {
  int32_t J[W];
  typename Vec2<T>::type k[W];
};

template <class T, int W>
__device__ inline void ell_load(int I, const int32_t* __restrict__ bcol_ell,
                                const T* __restrict__ B, int a, int b, EllRow<T, W>& e) {
  using V = typename Vec2<T>::type;
  const int64_t base = (int64_t)I * W;
  const int off = 6 * a + b;
  for (int u = 0; u < W; ++u) e.J[u] = bcol_ell[base + u];
  for (int u = 0; u < W; ++u) e.k[u] = *reinterpret_cast<const V*>(B + 36 * (base + u) + off);
}

// The three products over a loaded row: gathers of r, w, t at the row's columns.
template <class T, int W>
__device__ inline void ell_gather3(const EllRow<T, W>& e, const T* __restrict__ r,
                                   const T* __restrict__ w, const T* __restrict__ t, int b,
                                   T& ar, T& aw, T& at) {
  using V = typename Vec2<T>::type;
  const int32_t* J = e.J;
  const V* k = e.k;
  T sr = 0, sw = 0, st = 0;
  for (int u = 0; u < W; ++u) {
    const int64_t j = 6 * (int64_t)J[u] + b;
    const V rv = *reinterpret_cast<const V*>(r + j);
    const V wv = *reinterpret_cast<const V*>(w + j);
    const V tv = *reinterpret_cast<const V*>(t + j);
    sr += k[u].x * rv.x + k[u].y * rv.y;
    sw += k[u].x * wv.x + k[u].y * wv.y;
    st += k[u].x * tv.x + k[u].y * tv.y;
  }
  ar = sr;
  aw = sw;
  at = st;
}

template <class T, int W>
__device__ inline void row_product3_ell(int I, const int32_t* __restrict__ bcol_ell,
                                        const T* __restrict__ B, const T* __restrict__ r,
                                        const T* __restrict__ w, const T* __restrict__ t, int a,
                                        int b, T& ar, T& aw, T& at) {
  EllRow<T, W> e;
  ell_load<T, W>(I, bcol_ell, B, a, b, e);
  ell_gather3<T, W>(e, r, w, t, b, ar, aw, at);
}

// The state record seen through an address the compiler must treat as per-lane (offset by a
// zero it cannot see through), so its fields are fetched by vector loads issued with the other
// first-group loads and waited for where they are used, instead of by scalar loads that the
// kernel waits for before issuing anything else.
__device__ inline const PcgState* lane_view(const PcgState* st) {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return reinterpret_cast<const PcgState*>(reinterpret_cast<const char*>(st) + z);
}

// Single-vector product B x over the row (W = 0: block order of K via the row pointers).
template <class T, int W>
__device__ inline T row_product_b(const FusedDesc<T>& d, int I, const T* __restrict__ x, int a,
                                  int b) {
  if constexpr (W == 0) {
    return row_product<T, false>(d.brow_ptr, d.bcol, d.B, x, x, (T)0, I, a, b);
  } else {
    using V = typename Vec2<T>::type;
    const int64_t base = (int64_t)I * W;
    const int off = 6 * a + b;
    T acc = 0;
    for (int u = 0; u < W; ++u) {
      const int64_t J = d.bcol_ell[base + u];
      const V kv = *reinterpret_cast<const V*>(d.B + 36 * (base + u) + off);
      const V xv = *reinterpret_cast<const V*>(x + 6 * J + b);
      acc += kv.x * xv.x + kv.y * xv.y;
    }
    return acc;
  }
}

// Row a of the node's 6x6 block-Jacobi inverse (packed storage) applied to the 6 values at v.
// The 6 values v of this lane's node (SpMV layout: lane 18 g + 3 c of row group g holds
// component c), gathered by wave shuffles.
template <class T>
__device__ inline void node_values(T v, const SpLane& L, T out[6]) {
  const int base = ROW_LANES * L.g;
  for (int c = 0; c < 6; ++c) out[c] = __shfl(v, base + 3 * c, 64);
}

// x = 0, p = 0, r_0 = b, s_{-1} = 0; iteration counters and the state record reset.
template <class T>
__global__ void __launch_bounds__(MAX_TPB)
k_cg1_init1(const FusedDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob, double rtol,
            int max_it) {
  const WgOf<FusedDesc<T>> W = wg_of(D, wg_prob);
  const FusedDesc<T>& d = *W.d;
  const int64_t n_dof = 6 * (int64_t)d.n_nodes;
  for (int64_t q = (int64_t)W.lb * MAX_TPB + threadIdx.x; q < n_dof;
       q += (int64_t)W.ng * MAX_TPB) {
    d.x[q] = 0;
    d.p[q] = 0;
    d.r[0][q] = d.b[q];
    d.s[0][q] = 0;
  }
  if (threadIdx.x == 0) d.jw[W.lb] = 0;
  if (W.lb == 0 && threadIdx.x == 0) {
    PcgState* st = d.st;
    st->rtol2 = rtol * rtol;
    st->max_it = max_it;
    st->it = 0;
    st->done = 0;
    st->status = SSO_OK;
  }
}

// w_0 = B r_0; partials of gamma_0 = r_0.M r_0, delta_0 = w_0.M r_0, rho_0 = r_0.r_0.
template <class T, int W>
__global__ void __launch_bounds__(MAX_TPB)
k_cg1_init2(const FusedDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  __shared__ T rs[ROWS_PER_WG * 6];
  const WgOf<FusedDesc<T>> G = wg_of(D, wg_prob);
  const FusedDesc<T>& d = *G.d;
  const int n_nodes = d.n_nodes;
  const T* __restrict__ r0 = d.r[0];
  const SpLane L = sp_lane();
  const int slot = (threadIdx.x >> 6) * ROWS_PER_WAVE + L.g;
  T v[3] = {0, 0, 0};
  for (int gi = G.lb; gi * ROWS_PER_WG < n_nodes; gi += G.ng) {
    const int I = gi * ROWS_PER_WG + slot;
    const bool ok = L.ok && I < n_nodes;
    const bool own = ok && L.b == 0;
    const int64_t q = 6 * (int64_t)I + L.a;
    T acc = 0, rq = 0;
    if (ok) acc = row_product_b<T, W>(d, I, r0, L.a, L.b);
    const T wv = sum3(acc);
    if (own) {
      rq = r0[q];
      d.w[0][q] = wv;
      rs[6 * slot + L.a] = rq;
    }
    __syncthreads();
    if (own) {
      const T uq = dinv_row(d.Dinv, I, L.a).apply(rs + 6 * slot);
      v[0] += rq * uq;
      v[1] += wv * uq;
      v[2] += rq * rq;
    }
    __syncthreads();
  }
  block_sum<3, T>(v);
  write_partials<3, T>(v, d.pp[0], G.lb, G.ng);
}

// The operands of iteration i with the parity-dependent buffers resolved.  The host builds it
// for the single-problem kernel and passes it by value, so no kernel argument's address depends
// on another argument (the kernel issues its argument loads at once); multi-problem launches
// build it from the table entry and the workgroup's iteration counter.
template <class T>
struct Cg1Args {
  const T* r_in;
  const T* w_in;
  const T* s_in;
  T* r_out;
  T* w_out;
  T* s_out;
  T* p;
  T* x;
  const int32_t* brow_ptr;
  const int32_t* bcol;
  const int32_t* bcol_ell;
  const T* B;
  const T* Dinv;
  const double* pp_in;
  double* pp_out;
  PcgState* st;
  int32_t* jw;
  double rtol2;
  int n_nodes, i, max_it, n_wg;
};

template <class T>
__host__ __device__ inline Cg1Args<T> cg1_args(const FusedDesc<T>& d, int i) {
  Cg1Args<T> a;
  a.r_in = d.r[i & 1];
  a.w_in = d.w[i & 1];
  a.s_in = d.s[i & 1];
  a.r_out = d.r[(i + 1) & 1];
  a.w_out = d.w[(i + 1) & 1];
  a.s_out = d.s[(i + 1) & 1];
  a.p = d.p;
  a.x = d.x;
  a.brow_ptr = d.brow_ptr;
  a.bcol = d.bcol;
  a.bcol_ell = d.bcol_ell;
  a.B = d.B;
  a.Dinv = d.Dinv;
  a.pp_in = d.pp[i & 1];
  a.pp_out = d.pp[(i + 1) & 1];
  a.st = d.st;
  a.jw = d.jw;
  a.rtol2 = d.rtol2;
  a.n_nodes = d.n_nodes;
  a.i = i;
  a.max_it = d.max_it;
  a.n_wg = d.n_wg;
  return a;
}

// One single-reduction iteration for workgroup lb of ng.  SINGLE (one problem, launched by its
// own host loop): the iteration index comes from the host (launch k is iteration k until the
// state says done) and every load that does not depend on another -- done flag, state scalars,
// the previous partials, row pointers, own-row operands -- is issued before the done test, so
// an iteration costs three dependent memory round trips (row pointers, column indices and
// values, gathered vectors).  Otherwise (multi-problem launches) the index is the workgroup's
// own counter and the partials are loaded where they are summed, which keeps the register
// count, and the occupancy that many problems in flight need, lower.
template <class T, bool SINGLE, int W, bool ONE_PASS = false, bool JW = !SINGLE>
__device__ __forceinline__ void cg1_iteration(const Cg1Args<T>& d, int lb, int ng) {
  PcgState* st = d.st;
  const PcgState* stv = SINGLE ? lane_view(st) : st;
  const int done = stv->done;
  const int i = d.i;
  const int n_nodes = d.n_nodes;
  const T* __restrict__ ri = d.r_in;
  const T* __restrict__ wi = d.w_in;
  const T* __restrict__ so = d.s_in;
  T* __restrict__ rn = d.r_out;
  T* __restrict__ wn = d.w_out;
  T* __restrict__ sn = d.s_out;
  T* __restrict__ p = d.p;
  T* __restrict__ x = d.x;
  const SpLane L = sp_lane();
  const int slot = (threadIdx.x >> 6) * ROWS_PER_WAVE + L.g;
  // SINGLE: the state record through vector loads issued first, waited for with the rest of
  // the first group (the done test comes after the row's indices and values are issued)
  const double ff_prev = stv->ff, rtol2 = d.rtol2;
  const double gam_prev = stv->rzs[(i - 1) & 1], alpha_prev = stv->alphas[(i - 1) & 1];
  const int max_it = d.max_it;
  static_assert(3 * MAX_TPB >= PCG_MAX_WG, "three partials per thread");
  double pv[3][3] = {};
  T alpha = 0, beta = 0, ab = 0;
  T v[3] = {0, 0, 0};
  // ONE_PASS: the launch gives every workgroup rows (n_wg = ceil(n_nodes / 18)), so the body
  // runs once without an entry test and every kernel argument is loaded at once
  for (int gi = lb; ONE_PASS || gi * ROWS_PER_WG < n_nodes; gi += ng) {
    const int I = gi * ROWS_PER_WG + slot;
    const bool ok = L.ok && I < n_nodes;
    const bool own = ok && L.b == 0;
    const int64_t q = 6 * (int64_t)I + L.a;
    // loads without branches (lanes past the last row read row 0 and discard it), so that no
    // merge of a loaded register with a constant forces an early wait on the load
    const int Ic = ok ? I : 0;
    const int64_t qc = 6 * (int64_t)Ic + L.a;
    int rb = 0, re = 0;
    if constexpr (W == 0) {
      rb = d.brow_ptr[Ic];
      re = d.brow_ptr[Ic + 1];
    }
    T rq = 0, wq = 0, sq = 0, pq = 0, xq = 0;
    DinvRow<T> M{};
    if (SINGLE) {
      rq = ri[qc];
      wq = wi[qc];
      sq = so[qc];
      pq = p[qc];
      xq = x[qc];
      M = dinv_row(d.Dinv, Ic, L.a);
      // this thread's (at most 3) previous partials per sum, issued after the loads above so
      // that waiting for them waits for one round trip; added later in the order
      // finish_partials uses (ng <= PCG_MAX_WG <= 3 MAX_TPB); unconditional loads from a
      // clamped index, the out-of-range ones dropped where they are added
      if (gi == lb) {
        const double* pp = d.pp_in;
        for (int u = 0; u < 3; ++u) {
          const int k = (int)threadIdx.x + u * MAX_TPB;
          const int kc = k < ng ? k : 0;
          for (int c = 0; c < 3; ++c) pv[c][u] = pp[c * ng + kc];
        }
      }
    }
    T br = 0, bw = 0, bs = 0;
    if constexpr (W == 0) {
      if (!ok) re = rb;
      row_product3<T>(rb, re, d.bcol, d.B, ri, wi, so, L.a, L.b, br, bw, bs);
    } else {
      EllRow<T, W> e;
      ell_load<T, W>(Ic, d.bcol_ell, d.B, L.a, L.b, e);
      if (SINGLE && gi == lb) {
        // the column indices are in registers before the done test (their wait is the done
        // flag's, one round trip): a launch after convergence stops there, and the gathers
        // that depend on them go out right after it with the rest of the row's loads
        for (int u = 0; u < W; ++u) asm volatile("" ::"v"(e.J[u]));
        if (__builtin_amdgcn_readfirstlane(done)) return;
      }
      ell_gather3<T, W>(e, ri, wi, so, L.b, br, bw, bs);
    }
    if (!SINGLE) {
      rq = ri[qc];
      wq = wi[qc];
      sq = so[qc];
      pq = p[qc];
      xq = x[qc];
      M = dinv_row(d.Dinv, Ic, L.a);
    }
    if (gi == lb) {
      double tot[3];
      if (SINGLE) {
        const int k0 = (int)threadIdx.x;
        for (int c = 0; c < 3; ++c)
          tot[c] = ((0.0 + (k0 < ng ? pv[c][0] : 0.0)) +
                    (k0 + MAX_TPB < ng ? pv[c][1] : 0.0)) +
                   (k0 + 2 * MAX_TPB < ng ? pv[c][2] : 0.0);
        block_sum<3, double, 1, true>(tot);
        // block order of K: after the barrier of the sum, so that no load above is moved past
        // the test (a launch after convergence has read, in bounds, but writes nothing)
        if (W == 0 && __builtin_amdgcn_readfirstlane(done)) return;
      } else {
        finish_partials<3>(d.pp_in, ng, tot);
      }
      const double gam = tot[0], del = tot[1], rho = tot[2];
      const double ff = (i == 0) ? rho : ff_prev;
      double beta_d = 0.0, alpha_d;
      if (i == 0) {
        alpha_d = gam / del;
      } else {
        beta_d = gam / gam_prev;
        alpha_d = gam / (del - beta_d * gam / alpha_prev);
      }
      int stop = 0, status = SSO_OK;
      if (!std::isfinite(rho) || !std::isfinite(gam)) {
        stop = 1;
        status = SSO_EBREAKDOWN;
      } else if (rho <= rtol2 * ff) {
        stop = 1;
      } else if (i >= max_it) {
        stop = 1;
        status = SSO_ENOTCONV;
      } else if (!(alpha_d > 0.0) || !std::isfinite(alpha_d)) {
        stop = 1;
        status = SSO_EBREAKDOWN;
      }
      if (lb == 0 && threadIdx.x == 0) {
        st->rzs[i & 1] = gam;
        st->alphas[i & 1] = alpha_d;
        st->rr = rho;
        st->it = i;
        if (i == 0) st->ff = rho;
        if (stop) {
          st->status = status;
          st->done = 1;
        }
      }
      if (stop) return;
      alpha = (T)alpha_d;
      beta = (T)beta_d;
      ab = alpha * beta;
    }
    const T wv = sum3(br - alpha * bw - ab * bs);
    // every lane of a row holds its component a's operands; the node's 6 values of r_i and
    // r_{i+1} for M r come from the row's own lanes by wave shuffles (no LDS, no barrier)
    T r6[6];
    node_values(rq, L, r6);
    const T pv = M.apply(r6) + beta * pq;
    const T sv = wq + beta * sq;
    const T rv = rq - alpha * sv;
    // streaming stores: the next launch reads these from memory anyway (other XCDs), and
    // lines left dirty in this XCD's L2 would be written back at the kernel's end
    if (own) {
      __builtin_nontemporal_store(pv, &p[q]);
      __builtin_nontemporal_store(sv, &sn[q]);
      __builtin_nontemporal_store(xq + alpha * pv, &x[q]);
      __builtin_nontemporal_store(rv, &rn[q]);
      __builtin_nontemporal_store(wv, &wn[q]);
    }
    node_values(rv, L, r6);
    if (own) {
      const T uv = M.apply(r6);
      v[0] += rv * uv;
      v[1] += wv * uv;
      v[2] += rv * rv;
    }
    // one pass (the grid covers every row): no back edge, so the waits for the first group's
    // loads are placed where their values are used
    if constexpr (ONE_PASS) break;
  }
  block_sum<3, T, 2, true>(v);   // the kernel ends after it
  write_partials<3, T>(v, d.pp_out, lb, ng);
  if (JW && threadIdx.x == 0) d.jw[lb] = i + 1;
}

// Multi-problem form: descriptor table + workgroup map, iteration index per workgroup.
template <class T, int W>
__global__ void __launch_bounds__(MAX_TPB)
k_cg1_iter(const FusedDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  const WgOf<FusedDesc<T>> G = wg_of(D, wg_prob);
  if (G.d->st->done) return;
  cg1_iteration<T, false, W>(cg1_args(*G.d, G.d->jw[G.lb]), G.lb, G.ng);
}

// Multi-problem form for padded rows (W = 6, 9 or 12) with a register budget for many
// workgroups in flight: the iteration above, in the same arithmetic order, but with three slots a
// step (the next step's columns and values loaded with this step's gathers) instead of a whole
// row's loads at once, which holds the single-problem kernel to two waves per SIMD.  The
// descriptor is copied whole; the workgroup's iteration counter, the state, the first step's
// slots, the own-row operands and the previous partials (at most two per thread: n_wg <= 768)
// are issued together.  One pass: every row has a workgroup (n_wg x 18 >= n_nodes).
constexpr int CG1_LEAN_MAX_WG = 2 * MAX_TPB;

template <class T, int W>
__global__ void __launch_bounds__(MAX_TPB)
k_cg1_lean(const FusedDesc<T>* __restrict__ D, const int32_t* __restrict__ wg_prob) {
  static_assert(W % 3 == 0 && W > 0, "three padded slots a step");
  using V = typename Vec2<T>::type;
  const FusedDesc<T> d = D[wg_prob[blockIdx.x]];
  const int lb = (int)blockIdx.x - d.wg_base, ng = d.n_wg;
  const SpLane L = sp_lane();
  const int slot = (threadIdx.x >> 6) * ROWS_PER_WAVE + L.g;
  const int I = lb * ROWS_PER_WG + slot;
  const bool ok = L.ok && I < d.n_nodes;
  const bool own = ok && L.b == 0;
  const int Ic = ok ? I : 0;
  const int64_t q = 6 * (int64_t)I + L.a;
  const int64_t qc = 6 * (int64_t)Ic + L.a;
  // first group: iteration counter and state (vector loads, see lane_view), the first step's
  // slots, the own-row operands that do not depend on the iteration's parity, the inverse row,
  // the previous partials of both parities' buffers being unknown yet: read after the counter
  int zo;
  asm volatile("v_mov_b32 %0, 0" : "=v"(zo));
  const int i = __builtin_amdgcn_readfirstlane(
      *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(d.jw + lb) + zo));
  const PcgState* stv = lane_view(d.st);
  const int done = stv->done;
  const double ff_prev = stv->ff, rz0 = stv->rzs[0], rz1 = stv->rzs[1];
  const double al0 = stv->alphas[0], al1 = stv->alphas[1];
  const gptr<int32_t> bce = as_global(d.bcol_ell);
  const gptr<T> B = as_global(d.B);
  const int64_t base = (int64_t)Ic * W;
  const int off = 6 * L.a + L.b;
  int J[3];
  V kb[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    J[u] = bce[base + u];
    kb[u] = load2<V>(B + 36 * (base + u) + off);
  }
  const T pq = as_global(d.p)[qc], xq = as_global(d.x)[qc];
  if (__builtin_amdgcn_readfirstlane(done)) return;
  const int par = i & 1;
  // parity by selects: an array member indexed at run time would put the descriptor in scratch
  const gptr<T> ri = as_global(par ? d.r[1] : d.r[0]);
  const gptr<T> wi = as_global(par ? d.w[1] : d.w[0]);
  const gptr<T> so = as_global(par ? d.s[1] : d.s[0]);
  const gptr<double> pp = as_global(par ? d.pp[1] : d.pp[0]);
  const T rq = ri[qc], wq = wi[qc], sq = so[qc];
  double pv[3][2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int k = (int)threadIdx.x + u * MAX_TPB;
    const int kc = k < ng ? k : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[c][u] = pp[c * ng + kc];
  }
  T br = 0, bw = 0, bs = 0;
#pragma unroll 1
  for (int u0 = 0; u0 < W; u0 += 3) {
    V rv[3], wv[3], tv[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int64_t j = 6 * (int64_t)J[u] + L.b;
      rv[u] = load2<V>(ri + j);
      wv[u] = load2<V>(wi + j);
      tv[u] = load2<V>(so + j);
    }
    const int un = u0 + 3 < W ? u0 + 3 : u0;   // past the row: this step's slots again, unused
    int Jn[3];
    V kn[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      Jn[u] = bce[base + un + u];
      kn[u] = load2<V>(B + 36 * (base + un + u) + off);
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      br += kb[u].x * rv[u].x + kb[u].y * rv[u].y;
      bw += kb[u].x * wv[u].x + kb[u].y * wv[u].y;
      bs += kb[u].x * tv[u].x + kb[u].y * tv[u].y;
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      J[u] = Jn[u];
      kb[u] = kn[u];
    }
  }
  const DinvRow<T> M = dinv_row(d.Dinv, Ic, L.a);   // in flight across the reduction
  // the previous partials in the order of the single-problem iteration (a third per thread that
  // n_wg <= 768 never has), then the step lengths and the stopping test
  double tot[3];
  {
    const int k0 = (int)threadIdx.x;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      tot[c] = ((0.0 + (k0 < ng ? pv[c][0] : 0.0)) + (k0 + MAX_TPB < ng ? pv[c][1] : 0.0)) + 0.0;
  }
  block_sum<3, double, 1, true>(tot);
  const double gam = tot[0], del = tot[1], rho = tot[2];
  const double ff = (i == 0) ? rho : ff_prev;
  const double gam_prev = ((i - 1) & 1) ? rz1 : rz0, alpha_prev = ((i - 1) & 1) ? al1 : al0;
  double beta_d = 0.0, alpha_d;
  if (i == 0) {
    alpha_d = gam / del;
  } else {
    beta_d = gam / gam_prev;
    alpha_d = gam / (del - beta_d * gam / alpha_prev);
  }
  int stop = 0, status = SSO_OK;
  if (!std::isfinite(rho) || !std::isfinite(gam)) {
    stop = 1;
    status = SSO_EBREAKDOWN;
  } else if (rho <= d.rtol2 * ff) {
    stop = 1;
  } else if (i >= d.max_it) {
    stop = 1;
    status = SSO_ENOTCONV;
  } else if (!(alpha_d > 0.0) || !std::isfinite(alpha_d)) {
    stop = 1;
    status = SSO_EBREAKDOWN;
  }
  PcgState* st = d.st;
  if (lb == 0 && threadIdx.x == 0) {
    st->rzs[i & 1] = gam;
    st->alphas[i & 1] = alpha_d;
    st->rr = rho;
    st->it = i;
    if (i == 0) st->ff = rho;
    if (stop) {
      st->status = status;
      st->done = 1;
    }
  }
  if (stop) return;
  const T alpha = (T)alpha_d, beta = (T)beta_d, ab = alpha * beta;
  const T wv = sum3(br - alpha * bw - ab * bs);
  T r6[6];
  node_values(rq, L, r6);
  const T pvv = M.apply(r6) + beta * pq;
  const T sv = wq + beta * sq;
  const T rv = rq - alpha * sv;
  T v[3] = {0, 0, 0};
  T* const s_out = par ? d.s[0] : d.s[1];
  T* const r_out = par ? d.r[0] : d.r[1];
  T* const w_out = par ? d.w[0] : d.w[1];
  if (own) {
    __builtin_nontemporal_store(pvv, &d.p[q]);
    __builtin_nontemporal_store(sv, &s_out[q]);
    __builtin_nontemporal_store(xq + alpha * pvv, &d.x[q]);
    __builtin_nontemporal_store(rv, &r_out[q]);
    __builtin_nontemporal_store(wv, &w_out[q]);
  }
  node_values(rv, L, r6);
  if (own) {
    const T uv = M.apply(r6);
    v[0] += rv * uv;
    v[1] += wv * uv;
    v[2] += rv * rv;
  }
  block_sum<3, T, 2, true>(v);
  write_partials<3, T>(v, par ? d.pp[0] : d.pp[1], lb, ng);
  if (threadIdx.x == 0) d.jw[lb] = i + 1;
}

// One problem: the descriptor by value, launch k performs iteration k (unless done).
template <class T, int W, bool ONE_PASS>
__global__ void __launch_bounds__(MAX_TPB)
k_cg1_iter1(PcgState* st, const int32_t* bcol_ell, const T* B, const double* pp_in,
            const T* r_in, int n_nodes, int i, int n_wg, int max_it, Cg1Args<T> a) {
  // The leading scalar arguments arrive preloaded in SGPRs (14 dwords here; an aggregate
  // argument is not preloaded): what the first group of loads needs before the gathers, so they
  // go out without waiting for the argument segment.  The struct carries the rest.  Measured
  // against the struct alone: 60 x 60 / 80 x 80 / 40 x 40 shells 12.42 / 32.44 / 9.38 against
  // 12.73 / 32.96 / 9.69 ms per forward solve.
  a.st = st;
  a.bcol_ell = bcol_ell;
  a.B = B;
  a.pp_in = pp_in;
  a.r_in = r_in;
  a.n_nodes = n_nodes;
  a.i = i;
  a.max_it = max_it;
  a.n_wg = n_wg;
  // the grid is a.n_wg workgroups; taking the count from the arguments keeps it in the one
  // batch of argument loads
  cg1_iteration<T, true, W, ONE_PASS>(a, blockIdx.x, a.n_wg);
}

// Kernel of a padded width (0: block order of K); a width the pattern builder does not make is
// an error.
#define SSO_ELL_DISPATCH(W, CALL) \
  switch (W) {                    \
    case 0: CALL(0); break;       \
    case 6: CALL(6); break;       \
    case 9: CALL(9); break;       \
    case 12: CALL(12); break;     \
    default: return hipErrorInvalidValue; \
  }

// B = K M: block (I, J) of K times the block-Jacobi inverse of node J, one entry per thread, in
// the padded block-row layout (row I, slot u at (I w + u) 36; zero blocks past the row's count)
// or, with w = 0, in the block order of K.
template <class T>
__global__ void __launch_bounds__(256)
k_right_precondition(int n_nodes, int64_t n_blocks, int w, const int32_t* __restrict__ brow_ptr,
                     const int32_t* __restrict__ bcol, const double* __restrict__ K,
                     const double* __restrict__ Dinv, T* __restrict__ B) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n_out = w ? 36 * (int64_t)n_nodes * w : 36 * n_blocks;
  if (e >= n_out) return;
  const int64_t g = e / 36;   // output block
  const int ab = (int)(e - 36 * g), a = ab / 6, b = ab - 6 * a;
  int64_t s = g;              // block slot of K
  if (w) {
    const int I = (int)(g / w), u = (int)(g - (int64_t)I * w);
    const int rb = brow_ptr[I];
    if (u >= brow_ptr[I + 1] - rb) {
      B[e] = (T)0;
      return;
    }
    s = rb + u;
  }
  const double* k = K + 36 * s + 6 * a;
  const double* m = Dinv + DINV_PACKED * (int64_t)bcol[s];
  double acc = 0.0;
  for (int c = 0; c < 6; ++c) acc += k[c] * m[dinv_index(c, b)];
  B[e] = (T)acc;
}

// ---- compensated residual ------------------------------------------------------------------
// The true residual b - K x is a difference of nearly equal quantities: on a system whose
// products K_ij x_j are kappa times larger than the load, an FP64 evaluation carries a rounding
// error near kappa * eps relative to |b| (about 1.3e-10 on the 300 x 300 shell), so a residual
// target below that cannot be confirmed.  Here every product is split exactly with an FMA
// (two-product) and the sums are carried as unevaluated pairs hi + lo (two-sum), i.e. the row
// sum is formed in double-double arithmetic and rounded to FP64 once, after the subtraction
// from b.  Contraction is switched off so that the error terms are computed as written.

// s + e = a + b exactly (Knuth's two-sum).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += k * x, the product's rounding error recovered by an FMA.
__device__ __forceinline__ void dd_add_product(double k, double x, double& hi, double& lo) {
#pragma clang fp contract(off)
  const double p = k * x;
  const double pe = __builtin_fma(k, x, -p);
  double s, e;
  two_sum(hi, p, s, e);
  hi = s;
  lo += e + pe;
}

// (hi, lo) += (h2, l2).
__device__ __forceinline__ void dd_add(double h2, double l2, double& hi, double& lo) {
#pragma clang fp contract(off)
  double s, e;
  two_sum(hi, h2, s, e);
  hi = s;
  lo += e + l2;
}

// The row product of row_product<double, false> in double-double: this lane's entries (a,
// b..b+1) of every block of block row I against x.
__device__ inline void row_product_dd(const int32_t* __restrict__ brow_ptr,
                                      const int32_t* __restrict__ bcol,
                                      const double* __restrict__ K, const double* __restrict__ x,
                                      int I, int a, int b, double& hi, double& lo) {
  const int rb = brow_ptr[I], re = brow_ptr[I + 1];
  const int off = 6 * a + b;
  hi = 0.0;
  lo = 0.0;
  for (int s = rb; s < re; ++s) {
    const int64_t J = bcol[s];
    const double2 kv = *reinterpret_cast<const double2*>(K + 36 * (int64_t)s + off);
    const double2 xv = *reinterpret_cast<const double2*>(x + 6 * J + b);
    dd_add_product(kv.x, xv.x, hi, lo);
    dd_add_product(kv.y, xv.y, hi, lo);
  }
}

// r = b - K x with the row sums in double-double (rounded once); partials of ||r||^2 and
// ||b||^2.
__global__ void __launch_bounds__(MAX_TPB)
k_residual(int n_nodes, const int32_t* __restrict__ brow_ptr, const int32_t* __restrict__ bcol,
           const double* __restrict__ K, const double* __restrict__ x,
           const double* __restrict__ b, double* __restrict__ r, double* partials) {
#pragma clang fp contract(off)
  const SpLane L = sp_lane();
  const int wave = threadIdx.x >> 6;
  double v[2] = {0.0, 0.0};
  for (int gi = blockIdx.x; gi * ROWS_PER_WG < n_nodes; gi += gridDim.x) {
    const int I = gi * ROWS_PER_WG + wave * ROWS_PER_WAVE + L.g;
    const bool ok = L.ok && I < n_nodes;
    double hi = 0.0, lo = 0.0;
    if (ok) row_product_dd(brow_ptr, bcol, K, x, I, L.a, L.b, hi, lo);
    // the 3-lane set's pairs into its first lane (lane i reads lane i + 1), fixed order
    const double h1 = dpp_move<0x130>(hi), l1 = dpp_move<0x130>(lo);
    const double h2 = dpp_move<0x130>(h1), l2 = dpp_move<0x130>(l1);
    dd_add(h1, l1, hi, lo);
    dd_add(h2, l2, hi, lo);
    if (ok && L.b == 0) {
      const int64_t d = 6 * (int64_t)I + L.a;
      double s, e;
      two_sum(b[d], -hi, s, e);
      const double rv = s + (e - lo);
      if (r) r[d] = rv;
      v[0] += rv * rv;
      v[1] += b[d] * b[d];
    }
  }
  block_sum<2, double>(v);
  write_partials<2, double>(v, partials);
}

__global__ void __launch_bounds__(256)
k_dot(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* partials) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  double v[1] = {s};
  block_sum<1, double>(v);
  write_partials<1, double>(v, partials);
}

// One workgroup: out[k] = sum of partials array k (nv arrays of n), fixed order.
__global__ void __launch_bounds__(256) k_finish(const double* partials, int n, int nv,
                                                double* out) {
  double tot[2] = {0.0, 0.0};
  if (nv == 1) {
    finish_partials<1>(partials, n, tot);
  } else {
    finish_partials<2>(partials, n, tot);
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < nv; ++k) out[k] = tot[k];
}

// Copy the state records of a multi-problem launch into one array (one read-back per poll).
__global__ void k_gather_states(PcgState* const* st, int n, PcgState* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *st[i];
}

// y += alpha x
__global__ void k_axpy(int64_t n, double alpha, const double* x, double* y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}

__global__ void k_convert_f32(int64_t n, const double* in, float* out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// out = (float)(in * scale): the FP64 residual, normalised, as the FP32 inner right-hand side.
__global__ void k_scale_to_f32(int64_t n, const double* in, double scale, float* out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(in[i] * scale);
}

// ---- FP64 flexible CG around the FP32 inner solves ----------------------------------------
// Scalars (device, written by k_finish): sc[0] = r^T r, sc[2] = z^T q_prev, sc[3] = p^T q
// (the last direction's), sc[4] = p^T r.

// z = s * (double)d: the inner FP32 solution of K d = r / |r|, scaled back; partials of z^T q
// (the previous direction's product) when dot is set.
__global__ void __launch_bounds__(256)
k_fcg_z(int64_t n, double s, const float* __restrict__ d, const double* __restrict__ q,
        double* __restrict__ z, int dot, double* partials) {
  double v[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = s * (double)d[i];
    z[i] = zi;
    if (dot) v[0] += zi * q[i];
  }
  block_sum<1, double>(v);
  write_partials<1, double>(v, partials);
}

// p = z - beta p_prev with beta = z^T q_prev / p_prev^T q_prev (0 on a restart), q = K p with
// the direction formed on the fly from z and p_prev at the neighbour columns (p_prev and p are
// different buffers); partials of p^T q and p^T r.
__global__ void __launch_bounds__(MAX_TPB)
k_fcg_direction(int n_nodes, const int32_t* __restrict__ brow_ptr,
                const int32_t* __restrict__ bcol, const double* __restrict__ K,
                const double* __restrict__ z, const double* __restrict__ p_prev,
                const double* __restrict__ r, const double* __restrict__ sc, int restart,
                double* __restrict__ p, double* __restrict__ q, double* partials) {
  const SpLane L = sp_lane();
  const int wave = threadIdx.x >> 6;
  const double nb = restart ? 0.0 : -(sc[2] / sc[3]);
  double v[2] = {0.0, 0.0};
  for (int gi = blockIdx.x; gi * ROWS_PER_WG < n_nodes; gi += gridDim.x) {
    const int I = gi * ROWS_PER_WG + wave * ROWS_PER_WAVE + L.g;
    const bool ok = L.ok && I < n_nodes;
    double acc = 0.0;
    // on a (re)start p_prev is not read at all (it may hold anything)
    if (ok)
      acc = restart ? row_product<double, false>(brow_ptr, bcol, K, z, z, 0.0, I, L.a, L.b)
                    : row_product<double, true>(brow_ptr, bcol, K, z, p_prev, nb, I, L.a, L.b);
    const double sum = sum3(acc);
    if (ok && L.b == 0) {
      const int64_t d = 6 * (int64_t)I + L.a;
      const double pv = restart ? z[d] : z[d] + nb * p_prev[d];
      p[d] = pv;
      q[d] = sum;
      v[0] += pv * sum;
      v[1] += pv * r[d];
    }
  }
  block_sum<2, double>(v);
  write_partials<2, double>(v, partials);
}

// alpha = p^T r / p^T q (0 unless p^T q > 0); x += alpha p, r -= alpha q; partials of r^T r.
__global__ void __launch_bounds__(256)
k_fcg_update(int64_t n, const double* __restrict__ sc, const double* __restrict__ p,
             const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
             double* partials) {
  const double alpha = sc[3] > 0.0 ? sc[4] / sc[3] : 0.0;
  double v[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    v[0] += ri * ri;
  }
  block_sum<1, double>(v);
  write_partials<1, double>(v, partials);
}

}  // namespace

// Workgroups of a PCG launch: one pass of 18 block rows each, at most PCG_MAX_WG (every
// workgroup re-reads all partials of the previous launch, so their number bounds that cost);
// grid-stride beyond.  Measured on the 300 x 300 shell: 1024 workgroups beat a grid sized to
// one resident round of workgroups (occupancy x compute units) by 18 %.
static int choose_wg(int64_t n_nodes, int cap) {
  int64_t g = (n_nodes + ROWS_PER_WG - 1) / ROWS_PER_WG;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

// Passes over its rows that a workgroup of the standard recurrences makes at least (below the
// cap of PCG_MAX_WG workgroups): more passes amortise each workgroup's fixed start (descriptor,
// state, the previous kernel's partials) over more rows.  Measured (served stream closed loop
// of 256 requests / single 120 x 120 / single 300 x 300 shell): 1 pass 80.1 solves/s / 62.9 ms /
// 599.6 ms; 2 passes 93.1 / 62.6 / 606.3; 4 passes 94.1 / 85.1 / 590.8; 8 passes 89.9 / 137.9 /
// 674.3.  (The 300 x 300 shell is at the cap in every case.)  With three blocks per step in
// large multi-problem launches, 3 or 4 passes for problems of at most 8,192 nodes only (whose
// single solves take the fused kernel) gave 116.5 and 113.3 against 117.5-117.9 solves/s on
// 1,000 requests of the stream.
#ifndef SSO_STD_PASSES
#define SSO_STD_PASSES 2
#endif

// Workgroups of k_update that own nodes: it covers 64 nodes a pass where k_spmv_dir covers 36
// rows (two passes of 18), so of the n_wg workgroups that share the partial sums only the first
// ceil(n / 64) have work.  The others would write zero partials, which the initialisation kernel
// (all n_wg workgroups) has already left in their slots, so the update launches only these.
static inline int update_wg(int n_wg, int64_t n_nodes) {
  const int64_t g = (n_nodes + VEC_NODES - 1) / VEC_NODES;
  return (int)(g < n_wg ? (g < 1 ? 1 : g) : n_wg);
}

// Partial-sum buffers (units of the stride S = max(n_wg, n_wg_f, 1024) doubles):
//   [0, S) pA | [S, 3S) pB | [3S, 5S) one-off reductions, then 8 scalars |
//   [5S + 8, 8S + 8) single-reduction even | [8S + 8, 11S + 8) single-reduction odd
static int partial_stride(const PcgWork& w) {
  const int n = w.n_wg > w.n_wg_f ? w.n_wg : w.n_wg_f;
  return n > 1024 ? n : 1024;
}
static size_t partial_total(const PcgWork& w) { return 11 * (size_t)partial_stride(w) + 16; }
static double* part_a(PcgWork& w) { return w.partials; }
static double* part_b(PcgWork& w) { return w.partials + partial_stride(w); }
static double* part_once(PcgWork& w) { return w.partials + 3 * (size_t)partial_stride(w); }
static double* part_fused(PcgWork& w, int k) {
  return w.partials + (5 + 3 * k) * (size_t)partial_stride(w) + 8;
}

hipError_t pcg_alloc(PcgWork& w, int64_t n_nodes, bool mixed, hipStream_t s) {
  w.n_dof = 6 * n_nodes;
  w.n_wg = choose_wg((n_nodes + SSO_STD_PASSES - 1) / SSO_STD_PASSES, PCG_MAX_WG);
  w.n_wg_f = choose_wg(n_nodes, PCG_MAX_WG);
  hipError_t e;
  if ((e = dev_alloc(&w.r, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.z, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.p[0], w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.p[1], w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.Ap, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.xc, w.n_dof, s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.rc, w.n_dof, s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.partials, (int64_t)partial_total(w), s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.st, 1, s)) != hipSuccess) return e;
  if ((e = dev_alloc(reinterpret_cast<PcgDesc<double>**>(&w.desc64), 1, s)) != hipSuccess)
    return e;
  if ((e = dev_alloc(reinterpret_cast<PcgDesc<float>**>(&w.desc32), 1, s)) != hipSuccess)
    return e;
  if ((e = dev_alloc(reinterpret_cast<FusedDesc<double>**>(&w.fdesc64), 1, s)) != hipSuccess)
    return e;
  if ((e = dev_alloc(reinterpret_cast<FusedDesc<float>**>(&w.fdesc32), 1, s)) != hipSuccess)
    return e;
  if ((e = dev_alloc(&w.jw, w.n_wg_f, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(w.st, 0, sizeof(PcgState), s)) != hipSuccess) return e;
  w.h_st = new PcgState();
  if (mixed) return pcg_alloc_mixed(w, s);
  return hipSuccess;
}

hipError_t pcg_alloc_mixed(PcgWork& w, hipStream_t s) {
  if (w.r32) return hipSuccess;
  hipError_t e;
  if ((e = dev_alloc(&w.r32, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.z32, w.n_dof , s)) != hipSuccess) return e;
  // (z, p) pairs of the standard recurrences: two floats per DOF
  if ((e = dev_alloc(&w.p32[0], 2 * w.n_dof, s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.p32[1], 2 * w.n_dof, s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.Ap32, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.x32, w.n_dof , s)) != hipSuccess) return e;
  if ((e = dev_alloc(&w.b32, w.n_dof , s)) != hipSuccess) return e;
  return hipSuccess;
}

void pcg_free(PcgWork& w, const Arena* owner, hipStream_t s) {
  dev_release(w.r, owner, s); dev_release(w.z, owner, s); dev_release(w.p[0], owner, s); dev_release(w.p[1], owner, s);
  dev_release(w.Ap, owner, s); dev_release(w.partials, owner, s); dev_release(w.st, owner, s);
  dev_release(w.xc, owner, s); dev_release(w.rc, owner, s);
  dev_release(w.fw[0], owner, s); dev_release(w.fw[1], owner, s); dev_release(w.fw32[0], owner, s); dev_release(w.fw32[1], owner, s);
  dev_release(w.jw, owner, s); dev_release(w.fdesc64, owner, s); dev_release(w.fdesc32, owner, s);
  dev_release(w.desc64, owner, s); dev_release(w.desc32, owner, s);
  delete w.h_st;
  if (w.h_ring) {
    (void)hipStreamSynchronize(s);   // the last polled chunk's read-back may still be queued
    (void)hipHostFree(w.h_ring);
  }
  for (auto& ev : w.poll_ev)
    if (ev) (void)hipEventDestroy(ev);
  dev_release(w.r32, owner, s); dev_release(w.z32, owner, s); dev_release(w.p32[0], owner, s); dev_release(w.p32[1], owner, s);
  dev_release(w.Ap32, owner, s); dev_release(w.x32, owner, s); dev_release(w.b32, owner, s);
  if (w.prof_ev) {
    for (int i = 0; i < 2 * w.prof_cap; ++i) (void)hipEventDestroy(w.prof_ev[i]);
    delete[] w.prof_ev;
  }
  w = PcgWork();
}

// K bytes from which the standard recurrences write their vectors with streaming stores: a K
// this large (the 300 x 300 shell's is 234 MB) streams through the caches every iteration, and
// stores that bypass them leave more room for the gathered vectors.
static constexpr double STREAM_STORE_K_BYTES = 128.0 * (1 << 20);

static constexpr int PROF_CAP = 1024;
static constexpr int FUSED_SPAN = 8;   // launches per timing sample of the fused iteration
static constexpr int STD_SPAN = 8;     // iterations per timing sample of the standard pair

// Launch iterations in chunks of growing size (8 .. 64), reading the state record back after
// each chunk; launch(e0, e1) enqueues one iteration, recording e0 (when not null) before the
// kernel that is profiled and e1 (when not null) after it.  A sample starts at every
// profile_every-th launch and spans `span` consecutive launches (span divides 8, so a sample
// never crosses a chunk); launches past convergence return at entry, so only samples that end
// below the iteration count are kept: their mean duration per launch goes to w.prof_us /
// w.prof_n.
template <class F>
static hipError_t run_polled(PcgWork& w, hipStream_t s, int max_it, int profile_every, int span,
                             const F& launch, int* iters, int* status) {
  hipError_t e;
  if (profile_every > 0 && !w.prof_ev) {
    w.prof_ev = new hipEvent_t[2 * PROF_CAP];
    for (int i = 0; i < 2 * PROF_CAP; ++i)
      if ((e = hipEventCreate(&w.prof_ev[i])) != hipSuccess) return e;
    w.prof_cap = PROF_CAP;
  }
  if (profile_every > 0 && profile_every < span) profile_every = span;
  if (!w.h_ring) {
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&w.h_ring), 2 * sizeof(PcgState),
                           hipHostMallocDefault)) != hipSuccess)
      return e;
    for (auto& ev : w.poll_ev)
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  }
  // Two state read-backs in flight: chunk c + 1 is enqueued before the host waits for chunk c's
  // state, so the GPU does not idle at a poll; the launches of the chunk enqueued after
  // convergence return at entry.
  int n_prof = 0;
  int64_t launched = 0, launched_prev = 0;
  int chunk = 8;
  // (iteration, log(r.r / b.b)) of the last polls, for the chunk size near convergence
  constexpr int HIST = 4;
  int hist_it[HIST] = {};
  double hist_lr[HIST] = {};
  int n_hist = 0;
  for (int c = 0;; ++c) {
    int next = chunk < 64 ? 2 * chunk : 64;   // size of the chunk after this one
    // launch k performs iteration k and the one with index max_it stops on the limit: no launch
    // past it is ever needed (an inner solve of a few iterations would otherwise enqueue the
    // rest of the first chunks for nothing); polling ends when the state says done or once
    // the launch at the limit has run
    if (launched + chunk > (int64_t)max_it + 1)
      chunk = launched > (int64_t)max_it ? 0 : (int)((int64_t)max_it + 1 - launched);
    for (int i = 0; i < chunk; ++i) {
      const int64_t gk = launched + i;
      const int64_t ph = profile_every > 0 ? gk % profile_every : -1;
      const bool first = ph == 0 && n_prof < w.prof_cap;
      const bool last = ph == span - 1 && n_prof < w.prof_cap;
      launch(first ? &w.prof_ev[2 * n_prof] : nullptr,
             last ? &w.prof_ev[2 * n_prof + 1] : nullptr);
      if (last) ++n_prof;
    }
    launched += chunk;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&w.h_ring[c & 1], w.st, sizeof(PcgState), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(w.poll_ev[c & 1], s)) != hipSuccess) return e;
    if (c > 0) {
      if ((e = hipEventSynchronize(w.poll_ev[(c - 1) & 1])) != hipSuccess) return e;
      const PcgState& prev = w.h_ring[(c - 1) & 1];
      // done, or every launch up to the limit has run (the state read after them is final)
      if (prev.done || launched_prev > (int64_t)max_it) {
        *w.h_st = prev;
        break;
      }
      // Near convergence, size the next chunk from the residual's rate of decrease over the
      // last polls, so that few launches are enqueued past the converging iteration (they
      // cost a round trip each).  Only the chunking changes: the iteration that stops is
      // decided on the device.
      if (prev.rr > 0.0 && prev.ff > 0.0 && prev.rtol2 > 0.0) {
        const double lr = std::log(prev.rr / prev.ff);
        const int old = n_hist < HIST ? 0 : n_hist % HIST;
        if (n_hist > 0 && prev.it > hist_it[old]) {
          const double rate = (lr - hist_lr[old]) / (double)(prev.it - hist_it[old]);
          if (rate < 0.0) {
            // iterations still needed beyond those already enqueued, plus a margin; chunks
            // stay multiples of 8 (a timing sample never straddles two chunks)
            const double need = (std::log(prev.rtol2) - lr) / rate;
            const double left = need - (double)(launched - prev.it) + 8.0;
            if (left < (double)next) next = left <= 8.0 ? 8 : 8 * (int)((left + 7.0) / 8.0);
          }
        }
        hist_it[n_hist % HIST] = prev.it;
        hist_lr[n_hist % HIST] = lr;
        ++n_hist;
      }
    }
    launched_prev = launched;
    chunk = next;
  }
  *iters = w.h_st->it;
  *status = w.h_st->done ? w.h_st->status : SSO_ENOTCONV;
  for (int i = 0; i < n_prof; ++i) {
    if ((int64_t)i * profile_every + span > *iters) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, w.prof_ev[2 * i], w.prof_ev[2 * i + 1]) == hipSuccess) {
      w.prof_us += 1000.0 * ms / span;
      ++w.prof_n;
    }
  }
  return hipSuccess;
}

// Upload the descriptor of a standard solve and run its initialisation kernel.
template <class T>
static hipError_t pcg_start(const Mesh& m, const Pattern& pat, const T* K, const T* Dinv,
                            const T* b, T* x, T* r, T* z, T* const p[2], T* Ap, double rtol,
                            int max_it, PcgWork& w, hipStream_t s, PcgDesc<T>* out) {
  PcgDesc<T> hd{};
  hd.brow_ptr = pat.brow_ptr;
  hd.bcol = pat.bcol;
  hd.bsym = pat.bsym;
  hd.K = K;
  hd.Dinv = Dinv;
  hd.b = b;
  hd.x = x;
  hd.r = r;
  hd.z = z;
  hd.p[0] = p[0];
  hd.p[1] = p[1];
  hd.Ap = Ap;
  hd.pa = part_a(w);
  hd.pb = part_b(w);
  hd.st = w.st;
  hd.n_nodes = m.n_nodes;
  hd.n_wg = w.n_wg;
  hd.wg_base = 0;
  hd.n_blocks = pat.n_blocks;
  hd.stream_stores = 36.0 * sizeof(T) * (double)pat.n_blocks >= STREAM_STORE_K_BYTES ? 1 : 0;
  if (out) *out = hd;
  PcgDesc<T>* dd = reinterpret_cast<PcgDesc<T>*>(sizeof(T) == 8 ? w.desc64 : w.desc32);
  hipError_t e = hipMemcpyAsync(dd, &hd, sizeof(hd), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pcg_init<T>, dim3(w.n_wg), dim3(MAX_TPB), 0, s, dd, nullptr, rtol,
                     max_it);
  return hipGetLastError();
}

// One standard PCG solve in precision T on (K, Dinv, b) -> x; a profiled sample spans one
// whole iteration (k_spmv_dir and k_update).
template <class T>
static hipError_t pcg_run(const Mesh& m, const Pattern& pat, const T* K, const T* Dinv,
                          const T* b, T* x, T* r, T* z, T* const p[2], T* Ap, double rtol,
                          int max_it, PcgWork& w, hipStream_t s, int* iters, int* status,
                          int profile_every) {
  PcgDesc<T> hd{};
  hipError_t e = pcg_start<T>(m, pat, K, Dinv, b, x, r, z, p, Ap, rtol, max_it, w, s, &hd);
  if (e != hipSuccess) return e;
  const int nwg = w.n_wg;
  const int nwg_upd = update_wg(nwg, m.n_nodes);
  const bool sym = sym_products<T>(pat);
  const PcgDesc<T>* dd =
      reinterpret_cast<const PcgDesc<T>*>(sizeof(T) == 8 ? w.desc64 : w.desc32);
  // the single-problem kernels, whose first group's fields arrive as preloaded arguments:
  // against the descriptor alone, 54.3 against 54.7 us per iteration on the 300 x 300 shell,
  // 17.9 against 18.25 us on the 120 x 120 one (two alternating runs each)
  auto launch = [&](hipEvent_t* e0, hipEvent_t* e1) {
    if (e0) (void)hipEventRecord(*e0, s);
    if (sym)
      hipLaunchKernelGGL((k_spmv_dir_single<T, spmv_sym_ok<T>()>), dim3(nwg), dim3(MAX_TPB), 0,
                         s, hd.brow_ptr, hd.st, (const double*)hd.pb, hd.n_nodes, hd.n_wg, dd);
    else
      hipLaunchKernelGGL((k_spmv_dir_single<T, false>), dim3(nwg), dim3(MAX_TPB), 0, s,
                         hd.brow_ptr, hd.st, (const double*)hd.pb, hd.n_nodes, hd.n_wg, dd);
    hipLaunchKernelGGL(k_update_single<T>, dim3(nwg_upd), dim3(MAX_TPB), 0, s, hd.n_nodes,
                       hd.n_wg, (const T*)hd.Ap, hd.r, hd.p[0], hd.p[1], (const double*)hd.pa,
                       hd.st, dd);
    if (e1) (void)hipEventRecord(*e1, s);
  };
  // a sample spans 8 back-to-back iterations (events between every pair would add their own
  // latency to the iteration they bracket)
  return run_polled(w, s, max_it, profile_every, STD_SPAN, launch, iters, status);
}

// Vectors of one single-reduction solve.
template <class T>
struct FusedBuffers {
  T* x;
  T* p;
  T* r[2];
  T* s[2];
  T* w[2];
};

// One single-problem iteration launch for the descriptor's padded width (the width was checked
// when the solve started: fused_start).
template <class T, bool P1>
static void launch_iter1_w(const FusedDesc<T>& hd, int nwg, int k, hipStream_t s) {
  Cg1Args<T> a = cg1_args(hd, k);
  a.n_wg = nwg;   // the grid launched below
  switch (hd.ell_w) {
    case 6:
      hipLaunchKernelGGL((k_cg1_iter1<T, 6, P1>), dim3(nwg), dim3(MAX_TPB), 0, s, a.st,
                         a.bcol_ell, a.B, a.pp_in, a.r_in, a.n_nodes, a.i, a.n_wg, a.max_it, a);
      break;
    case 9:
      hipLaunchKernelGGL((k_cg1_iter1<T, 9, P1>), dim3(nwg), dim3(MAX_TPB), 0, s, a.st,
                         a.bcol_ell, a.B, a.pp_in, a.r_in, a.n_nodes, a.i, a.n_wg, a.max_it, a);
      break;
    case 12:
      hipLaunchKernelGGL((k_cg1_iter1<T, 12, P1>), dim3(nwg), dim3(MAX_TPB), 0, s, a.st,
                         a.bcol_ell, a.B, a.pp_in, a.r_in, a.n_nodes, a.i, a.n_wg, a.max_it, a);
      break;
    default:
      hipLaunchKernelGGL((k_cg1_iter1<T, 0, P1>), dim3(nwg), dim3(MAX_TPB), 0, s, a.st,
                         a.bcol_ell, a.B, a.pp_in, a.r_in, a.n_nodes, a.i, a.n_wg, a.max_it, a);
  }
}

template <class T>
static void launch_iter1(const FusedDesc<T>& hd, int nwg, int k, hipStream_t s) {
  if ((int64_t)nwg * ROWS_PER_WG >= hd.n_nodes)
    launch_iter1_w<T, true>(hd, nwg, k, s);
  else
    launch_iter1_w<T, false>(hd, nwg, k, s);
}

template <class T>
static FusedDesc<T> fused_desc(const Mesh& m, const Pattern& pat, const T* B, const T* Dinv,
                               const T* b, const FusedBuffers<T>& v, PcgWork& w) {
  FusedDesc<T> hd{};
  hd.brow_ptr = pat.brow_ptr;
  hd.bcol = pat.bcol;
  hd.bcol_ell = pat.bcol_ell;
  hd.ell_w = pat.ell_w;
  hd.B = B;
  hd.Dinv = Dinv;
  hd.b = b;
  hd.x = v.x;
  hd.p = v.p;
  for (int k = 0; k < 2; ++k) {
    hd.r[k] = v.r[k];
    hd.s[k] = v.s[k];
    hd.w[k] = v.w[k];
    hd.pp[k] = part_fused(w, k);
  }
  hd.jw = w.jw;
  hd.st = w.st;
  hd.n_nodes = m.n_nodes;
  hd.n_wg = w.n_wg_f;
  hd.wg_base = 0;
  return hd;
}

// Upload the descriptor and start a single-reduction solve (initial residual and partials).
template <class T>
static hipError_t fused_start(FusedDesc<T>& hd, double rtol, int max_it, PcgWork& w,
                              hipStream_t s, FusedDesc<T>** out) {
  hd.rtol2 = rtol * rtol;
  hd.max_it = max_it;
  FusedDesc<T>* dd = reinterpret_cast<FusedDesc<T>*>(sizeof(T) == 8 ? w.fdesc64 : w.fdesc32);
  hipError_t e = hipMemcpyAsync(dd, &hd, sizeof(hd), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cg1_init1<T>, dim3(hd.n_wg), dim3(MAX_TPB), 0, s, dd, nullptr, rtol,
                     max_it);
#define SSO_INIT2(W) \
  hipLaunchKernelGGL((k_cg1_init2<T, W>), dim3(hd.n_wg), dim3(MAX_TPB), 0, s, dd, nullptr)
  SSO_ELL_DISPATCH(hd.ell_w, SSO_INIT2)
#undef SSO_INIT2
  *out = dd;
  return hipGetLastError();
}

// One single-reduction PCG solve in precision T with B = K Dinv; the iteration kernel (the
// whole iteration) is profiled.
template <class T>
static hipError_t fused_run(const Mesh& m, const Pattern& pat, const T* B, const T* Dinv,
                            const T* b, const FusedBuffers<T>& v, double rtol, int max_it,
                            PcgWork& w, hipStream_t s, int* iters, int* status,
                            int profile_every) {
  FusedDesc<T> hd = fused_desc(m, pat, B, Dinv, b, v, w);
  FusedDesc<T>* dd = nullptr;
  hipError_t e = fused_start(hd, rtol, max_it, w, s, &dd);
  if (e != hipSuccess) return e;
  const int nwg = hd.n_wg;
  int k = 0;   // launch index = iteration index until the state says done
  auto launch = [&](hipEvent_t* e0, hipEvent_t* e1) {
    if (e0) (void)hipEventRecord(*e0, s);
    launch_iter1(hd, nwg, k, s);
    if (e1) (void)hipEventRecord(*e1, s);
    ++k;
  };
  // the only kernel of an iteration: samples of 8 back-to-back launches
  return run_polled(w, s, max_it, profile_every, FUSED_SPAN, launch, iters, status);
}

static hipError_t fused_alloc(PcgWork& w, bool f32, hipStream_t s) {
  hipError_t e;
  for (int k = 0; k < 2; ++k) {
    if (!f32 && !w.fw[k] && (e = dev_alloc(&w.fw[k], w.n_dof, s)) != hipSuccess) return e;
    if (f32 && !w.fw32[k] && (e = dev_alloc(&w.fw32[k], w.n_dof, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t pcg_begin(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                     const double* b, double* x, double rtol, int max_it, PcgWork& w,
                     hipStream_t s, PcgDesc<double>* desc) {
  hipError_t e = pcg_start<double>(m, pat, K, Dinv, b, x, w.r, w.z, w.p, w.Ap, rtol, max_it, w,
                                   s, desc);
  w.h_st->done = 0;
  w.h_st->jn = 0;   // as k_pcg_init leaves the device state
  return e;
}

hipError_t fused_begin(const Mesh& m, const Pattern& pat, const double* B, const double* Dinv,
                       const double* b, double* x, double rtol, int max_it, PcgWork& w,
                       hipStream_t s, FusedDesc<double>* desc) {
  hipError_t e;
  if ((e = fused_alloc(w, false, s)) != hipSuccess) return e;
  const FusedBuffers<double> v{x, w.p[0], {w.r, w.z}, {w.p[1], w.Ap}, {w.fw[0], w.fw[1]}};
  *desc = fused_desc(m, pat, B, Dinv, b, v, w);
  FusedDesc<double>* dd = nullptr;
  if ((e = fused_start(*desc, rtol, max_it, w, s, &dd)) != hipSuccess) return e;
  w.h_st->done = 0;
  return hipSuccess;
}

// Lays the problems' workgroups out one problem after another (wg_base: the first of each) and
// uploads the descriptors and the workgroup -> problem map.  update: the k_update launch, which
// takes only the workgroups that own nodes (update_wg); n_wg stays the partial sums' count.
template <class Desc>
static hipError_t table_upload(LaunchTable<Desc>& t, const Desc* descs, int n, hipStream_t s,
                               bool update = false) {
  t.h_desc.assign(descs, descs + n);
  t.h_wg.clear();
  for (int i = 0; i < n; ++i) {
    t.h_desc[i].wg_base = (int)t.h_wg.size();
    const int nw =
        update ? update_wg(t.h_desc[i].n_wg, t.h_desc[i].n_nodes) : t.h_desc[i].n_wg;
    for (int k = 0; k < nw; ++k) t.h_wg.push_back(i);
  }
  t.total = (int)t.h_wg.size();
  if (n == 0) return hipSuccess;
  hipError_t e;
  if (n > t.cap_desc) {
    dev_free(t.d_desc, s);
    t.d_desc = nullptr;
    t.cap_desc = 2 * n;
    e = dev_alloc_scratch(reinterpret_cast<Desc**>(&t.d_desc), t.cap_desc, s);
    if (e != hipSuccess) return e;
  }
  if (t.total > t.cap_wg) {
    dev_free(t.d_wg, s);
    t.d_wg = nullptr;
    t.cap_wg = 2 * t.total;
    if ((e = dev_alloc_scratch(&t.d_wg, t.cap_wg, s)) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(t.d_desc, t.h_desc.data(), sizeof(Desc) * n, hipMemcpyHostToDevice,
                          s)) != hipSuccess)
    return e;
  return hipMemcpyAsync(t.d_wg, t.h_wg.data(), sizeof(int32_t) * t.total,
                        hipMemcpyHostToDevice, s);
}

template <class Desc>
static void table_free(LaunchTable<Desc>& t, hipStream_t s) {
  dev_free(t.d_desc, s);
  dev_free(t.d_wg, s);
}

// Multi-problem launches of more workgroups than stay resident at once run the product kernel
// with three blocks per step (74 VGPRs, 6 waves per SIMD): every workgroup there makes only a
// few passes, and more loads in flight per wave beat occupancy.  Measured on one box, 32 and
// 48 60 x 60 shells per launch: 3.32-3.35 against 3.41 and 3.30 against 3.38 us per problem-
// iteration; the served stream 114.7-114.8 against 112.3 solves/s.  Four per step (91 VGPRs,
// 5 waves) lost (3.8-3.9 us); single problems keep two (the 300 x 300 shell: bandwidth-bound).
constexpr int BATCH_NB = 3;
constexpr int BATCH_NB_MIN_WG = 1024;

template <class T>
static void launch_standard(const LaunchTable<PcgDesc<T>>& t, const LaunchTable<PcgDesc<T>>& u,
                            hipStream_t s) {
  if (t.total == 0) return;
  const PcgDesc<T>* d = reinterpret_cast<const PcgDesc<T>*>(t.d_desc);
  if constexpr (sizeof(T) == 8) {
    if (t.sym) {
      hipLaunchKernelGGL(k_spmv_dir_sym<T>, dim3(t.total), dim3(MAX_TPB), 0, s, d, t.d_wg);
      hipLaunchKernelGGL(k_update<T>, dim3(u.total), dim3(MAX_TPB), 0, s,
                         reinterpret_cast<const PcgDesc<T>*>(u.d_desc), u.d_wg);
      return;
    }
  }
  if (t.total > BATCH_NB_MIN_WG)
    hipLaunchKernelGGL((k_spmv_dir<T, BATCH_NB>), dim3(t.total), dim3(MAX_TPB), 0, s, d,
                       t.d_wg);
  else
    hipLaunchKernelGGL(k_spmv_dir<T>, dim3(t.total), dim3(MAX_TPB), 0, s, d, t.d_wg);
  hipLaunchKernelGGL(k_update<T>, dim3(u.total), dim3(MAX_TPB), 0, s,
                     reinterpret_cast<const PcgDesc<T>*>(u.d_desc), u.d_wg);
}

template <class T, int W>
static void launch_fused_w(const LaunchTable<FusedDesc<T>>& t, hipStream_t s) {
  const FusedDesc<T>* d = reinterpret_cast<const FusedDesc<T>*>(t.d_desc);
  if constexpr (W > 0) {
    if (t.lean) {
      hipLaunchKernelGGL((k_cg1_lean<T, W>), dim3(t.total), dim3(MAX_TPB), 0, s, d, t.d_wg);
      return;
    }
  }
  hipLaunchKernelGGL((k_cg1_iter<T, W>), dim3(t.total), dim3(MAX_TPB), 0, s, d, t.d_wg);
}

template <class T>
static void launch_fused(const std::map<int, LaunchTable<FusedDesc<T>>>& tables, hipStream_t s) {
  for (const auto& kv : tables) {
    if (kv.second.total == 0) continue;
    switch (kv.first) {
      case 6: launch_fused_w<T, 6>(kv.second, s); break;
      case 9: launch_fused_w<T, 9>(kv.second, s); break;
      case 12: launch_fused_w<T, 12>(kv.second, s); break;
      default: launch_fused_w<T, 0>(kv.second, s);
    }
  }
}

// Per padded width, the problems of one fused list laid into that width's table.
template <class T>
static hipError_t fused_upload(std::map<int, LaunchTable<FusedDesc<T>>>& tables,
                               const std::vector<FusedDesc<T>>& list, hipStream_t s) {
  std::map<int, std::vector<FusedDesc<T>>> by_w;
  for (const auto& d : list) by_w[d.ell_w].push_back(d);
  for (auto& kv : tables) kv.second.total = 0;
  for (const auto& kv : by_w) {
    if (kv.first != 0 && kv.first != 6 && kv.first != 9 && kv.first != 12 && kv.first != 16)
      return hipErrorInvalidValue;
    hipError_t e = table_upload(tables[kv.first], kv.second.data(), (int)kv.second.size(), s);
    if (e != hipSuccess) return e;
    bool lean = true;   // every problem one pass, at most CG1_LEAN_MAX_WG workgroups
    for (const auto& d : kv.second)
      lean = lean && d.n_wg <= CG1_LEAN_MAX_WG && (int64_t)d.n_wg * ROWS_PER_WG >= d.n_nodes;
    tables[kv.first].lean = lean;
  }
  return hipSuccess;
}

// A multi-problem launch gives each one-workgroup problem this many times the iterations of the
// other kinds (an iteration of a small problem on one workgroup takes a few microseconds, the
// launch pairs of the others a hundred or so when many problems are in flight).
constexpr int WG1_BATCH_FACTOR = 16;

// The one-workgroup problems' launch runs on a second stream of the batch, beside the launches
// of the other kinds: it waits for what the batch stream enqueued before it (the problems' own
// earlier work and the table upload), and the batch stream waits for it before the states are
// gathered.
static hipError_t launch_wg(BatchWork& bw, int n_iter, hipStream_t s) {
  const int np = bw.wg.total;
  if (np == 0) return hipSuccess;
  hipError_t e;
  if (!bw.s_wg) {
    int dev = 0, cur = 0;
    if ((e = hipStreamGetDevice(s, &dev)) != hipSuccess) return e;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    e = hipStreamCreateWithFlags(&bw.s_wg, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bw.ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bw.ev_wg, hipEventDisableTiming);
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
  }
  if ((e = hipEventRecord(bw.ev_in, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(bw.s_wg, bw.ev_in, 0)) != hipSuccess) return e;
  const int64_t budget = (int64_t)n_iter * WG1_BATCH_FACTOR;
  const int it = budget > (1 << 30) ? (1 << 30) : (int)budget;
  hipLaunchKernelGGL(k_pcg_wg, dim3(np), dim3(WG1_TPB), WGL_LDS_BYTES, bw.s_wg,
                     reinterpret_cast<const PcgDesc<double>*>(bw.wg.d_desc), it, WGL_LDS_BYTES);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipEventRecord(bw.ev_wg, bw.s_wg);
}

hipError_t pcg_batch_launch(const BatchLists& L, int n_iter, BatchWork& bw, hipStream_t s) {
  const int nt = (int)(L.standard.size() + L.fused.size() + L.standard32.size() +
                       L.fused32.size() + L.wg.size());
  bw.pending_nt = nt;
  if (nt <= 0) return hipSuccess;
  hipError_t e;
  if ((e = table_upload(bw.standard, L.standard.data(), (int)L.standard.size(), s)) !=
      hipSuccess)
    return e;
  {
    // the upper-triangle products once the problems' K together outgrow the Infinity Cache
    double kb = 0.0;
    for (const auto& d : L.standard) kb += 36.0 * 8.0 * (double)d.n_blocks;
    bw.standard.sym = kb >= SYM_PRODUCT_MIN_K_BYTES;
  }
  if ((e = table_upload(bw.standard_upd, L.standard.data(), (int)L.standard.size(), s, true)) !=
      hipSuccess)
    return e;
  if ((e = fused_upload(bw.fused, L.fused, s)) != hipSuccess) return e;
  if ((e = table_upload(bw.standard32, L.standard32.data(), (int)L.standard32.size(), s)) !=
      hipSuccess)
    return e;
  if ((e = table_upload(bw.standard32_upd, L.standard32.data(), (int)L.standard32.size(), s,
                        true)) != hipSuccess)
    return e;
  if ((e = fused_upload(bw.fused32, L.fused32, s)) != hipSuccess) return e;
  if ((e = table_upload(bw.wg, L.wg.data(), (int)L.wg.size(), s)) != hipSuccess) return e;
  if (n_iter > 0 && (e = launch_wg(bw, n_iter, s)) != hipSuccess) return e;
  const int span = bw.time_span < n_iter ? bw.time_span : n_iter;
  for (int i = 0; i < n_iter; ++i) {
    if (span > 0 && i == 0 && (e = hipEventRecord(bw.ev_t0, s)) != hipSuccess) return e;
    launch_standard(bw.standard, bw.standard_upd, s);
    launch_fused(bw.fused, s);
    launch_standard(bw.standard32, bw.standard32_upd, s);
    launch_fused(bw.fused32, s);
    ++bw.launched;
    if (span > 0 && i + 1 == span && (e = hipEventRecord(bw.ev_t1, s)) != hipSuccess) return e;
  }
  bw.h_stp.clear();
  for (const auto& d : L.standard) bw.h_stp.push_back(d.st);
  for (const auto& d : L.fused) bw.h_stp.push_back(d.st);
  for (const auto& d : L.standard32) bw.h_stp.push_back(d.st);
  for (const auto& d : L.fused32) bw.h_stp.push_back(d.st);
  for (const auto& d : L.wg) bw.h_stp.push_back(d.st);
  if (n_iter > 0 && bw.wg.total > 0 && (e = hipStreamWaitEvent(s, bw.ev_wg, 0)) != hipSuccess)
    return e;
  if (nt > bw.cap_states) {
    dev_free(bw.d_states, s);
    dev_free(bw.d_stp, s);
    bw.d_states = nullptr;
    bw.d_stp = nullptr;
    bw.cap_states = bw.cap_stp = 2 * nt;
    if ((e = dev_alloc_scratch(&bw.d_states, bw.cap_states, s)) != hipSuccess) return e;
    if ((e = dev_alloc_scratch(&bw.d_stp, bw.cap_stp, s)) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(bw.d_stp, bw.h_stp.data(), sizeof(PcgState*) * nt,
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_gather_states, dim3((nt + 63) / 64), dim3(64), 0, s, bw.d_stp, nt,
                     bw.d_states);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nt > bw.cap_pin) {   // no copy into the old buffer is pending: the last launch was waited for
    if (bw.h_pin) (void)hipHostFree(bw.h_pin);
    bw.h_pin = nullptr;
    bw.cap_pin = 0;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&bw.h_pin), sizeof(PcgState) * 2 * nt,
                           hipHostMallocDefault)) != hipSuccess)
      return e;
    bw.cap_pin = 2 * nt;
  }
  if (!bw.ev && (e = hipEventCreateWithFlags(&bw.ev, hipEventDisableTiming)) != hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(bw.h_pin, bw.d_states, sizeof(PcgState) * nt, hipMemcpyDeviceToHost,
                          s)) != hipSuccess)
    return e;
  return hipEventRecord(bw.ev, s);
}

hipError_t pcg_batch_wait(BatchWork& bw) {
  const int nt = bw.pending_nt;
  bw.pending_nt = -1;
  if (nt <= 0) {
    bw.h_states.clear();
    return hipSuccess;
  }
  hipError_t e = hipEventSynchronize(bw.ev);
  if (e != hipSuccess) return e;
  bw.h_states.assign(bw.h_pin, bw.h_pin + nt);
  return hipSuccess;
}

hipError_t pcg_batch_iterate(const BatchLists& L, int n_iter, BatchWork& bw, hipStream_t s) {
  hipError_t e = pcg_batch_launch(L, n_iter, bw, s);
  if (e != hipSuccess) return e;
  return pcg_batch_wait(bw);
}

void batch_free(BatchWork& bw, hipStream_t s) {
  if (bw.ev) {
    (void)hipEventSynchronize(bw.ev);
    (void)hipEventDestroy(bw.ev);
  }
  if (bw.h_pin) (void)hipHostFree(bw.h_pin);
  table_free(bw.standard, s);
  for (auto& kv : bw.fused) table_free(kv.second, s);
  table_free(bw.standard32, s);
  for (auto& kv : bw.fused32) table_free(kv.second, s);
  table_free(bw.wg, s);
  table_free(bw.standard_upd, s);
  table_free(bw.standard32_upd, s);
  if (bw.s_wg) {
    (void)hipStreamSynchronize(bw.s_wg);
    (void)hipStreamDestroy(bw.s_wg);
  }
  if (bw.ev_in) (void)hipEventDestroy(bw.ev_in);
  if (bw.ev_wg) (void)hipEventDestroy(bw.ev_wg);
  if (bw.ev_t0) (void)hipEventDestroy(bw.ev_t0);
  if (bw.ev_t1) (void)hipEventDestroy(bw.ev_t1);
  dev_free(bw.d_stp, s);
  dev_free(bw.d_states, s);
  bw = BatchWork();
}

// Up to this many nodes the single launch per iteration of the single-reduction recurrences wins
// (the 60 x 60 shell: 13.4 vs 20.2 ms per solve); from about 8,000 nodes the standard pair is as
// fast or faster (90 x 90: 46.2 vs 45.3 ms; 120 x 120: 88 vs 63 ms), and on large problems it
// streams closer to the bandwidth peak (the 300 x 300 shell: 80 vs 125 us per iteration).
static constexpr int64_t FUSED_MAX_NODES = 8192;
static_assert(FUSED_MAX_NODES <= (int64_t)PCG_MAX_WG * ROWS_PER_WG,
              "the single-reduction recurrences run in one pass of the grid");

// AUTO: one workgroup per problem (FP64) when the problem is resident in its LDS (at most 144 nodes;
// single solves measured 1.50 against 2.87 ms at 64 nodes, 3.07 against 4.39 ms at 121 and
// 2.67 against 3.26 ms at 144), the single-reduction recurrences up to FUSED_MAX_NODES, the
// standard ones above.
int pcg_pick_solver(int solver, int64_t n_nodes, int64_t n_blocks, bool mixed) {
  if (solver == SSO_SOLVER_STANDARD || solver == SSO_SOLVER_FUSED || solver == SSO_SOLVER_WG)
    return solver;
  if (!mixed && n_nodes <= WGL_MAX_NODES && wgl_bytes(n_nodes, n_blocks) <= WGL_LDS_BYTES)
    return SSO_SOLVER_WG;
  return n_nodes <= FUSED_MAX_NODES ? SSO_SOLVER_FUSED : SSO_SOLVER_STANDARD;
}

int64_t right_precondition_blocks(const Pattern& pat, int64_t n_nodes) {
  return pat.ell_w ? n_nodes * pat.ell_w : pat.n_blocks;
}

hipError_t launch_right_precondition(const Mesh& m, const Pattern& pat, const double* K,
                                     const double* Dinv, double* B, float* B32, hipStream_t s) {
  const int64_t n = 36 * right_precondition_blocks(pat, m.n_nodes);
  if (B)
    hipLaunchKernelGGL(k_right_precondition<double>, dim3(nblk(n, 256)), dim3(256), 0, s,
                       m.n_nodes, pat.n_blocks, pat.ell_w, pat.brow_ptr, pat.bcol, K, Dinv, B);
  if (B32)
    hipLaunchKernelGGL(k_right_precondition<float>, dim3(nblk(n, 256)), dim3(256), 0, s,
                       m.n_nodes, pat.n_blocks, pat.ell_w, pat.brow_ptr, pat.bcol, K, Dinv,
                       B32);
  return hipGetLastError();
}

// Iterations per launch of a single solve on one workgroup (k_pcg_wg): a solve of up to this
// many iterations is one launch.
constexpr int WG1_SOLO_ITERS = 1 << 14;

hipError_t pcg_solve_wg(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                        const double* b, double* x, double rtol, int max_it, PcgWork& w,
                        hipStream_t s, int* iters, int* status, int profile_every) {
  w.prof_us = 0.0;
  w.prof_n = 0;
  hipError_t e = pcg_start<double>(m, pat, K, Dinv, b, x, w.r, w.z, w.p, w.Ap, rtol, max_it, w,
                                   s, nullptr);
  if (e != hipSuccess) return e;
  if (profile_every > 0 && !w.prof_ev) {
    w.prof_ev = new hipEvent_t[2 * PROF_CAP];
    for (int i = 0; i < 2 * PROF_CAP; ++i)
      if ((e = hipEventCreate(&w.prof_ev[i])) != hipSuccess) return e;
    w.prof_cap = PROF_CAP;
  }
  const PcgDesc<double>* dd = reinterpret_cast<const PcgDesc<double>*>(w.desc64);
  // resident in LDS when the problem fits
  const int64_t lb = wgl_bytes(m.n_nodes, pat.n_blocks);
  const int lds = (m.n_nodes <= WGL_MAX_NODES && lb <= WGL_LDS_BYTES) ? (int)lb : 0;
  // the kernel stops itself at iteration max_it, so the launches end
  for (int64_t launched = 0;; launched += WG1_SOLO_ITERS) {
    const bool prof = profile_every > 0 && launched == 0;
    if (prof && (e = hipEventRecord(w.prof_ev[0], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pcg_wg, dim3(1), dim3(WG1_TPB), lds, s, dd, WG1_SOLO_ITERS, lds);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (prof && (e = hipEventRecord(w.prof_ev[1], s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(w.h_st, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (prof && w.h_st->it > 0) {   // mean duration of an iteration of the first launch
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, w.prof_ev[0], w.prof_ev[1]) == hipSuccess) {
        w.prof_us = 1000.0 * ms / w.h_st->it;
        w.prof_n = 1;
      }
    }
    if (w.h_st->done) break;
  }
  *iters = w.h_st->it;
  *status = w.h_st->status;
  if (*status != SSO_OK) return hipSuccess;
  return pcg_correct(m, pat, K, Dinv, b, x, rtol, max_it, w, s, iters, status);
}

hipError_t pcg_solve(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                     const double* B, const double* b, double* x, double rtol, int max_it,
                     PcgWork& w, hipStream_t s, int* iters, int* status, int profile_every) {
  w.prof_us = 0.0;
  w.prof_n = 0;
  hipError_t e;
  if (B) {
    if ((e = fused_alloc(w, false, s)) != hipSuccess) return e;
    const FusedBuffers<double> v{x, w.p[0], {w.r, w.z}, {w.p[1], w.Ap}, {w.fw[0], w.fw[1]}};
    e = fused_run<double>(m, pat, B, Dinv, b, v, rtol, max_it, w, s, iters, status,
                          profile_every);
  } else {
    e = pcg_run<double>(m, pat, K, Dinv, b, x, w.r, w.z, w.p, w.Ap, rtol, max_it, w, s, iters,
                        status, profile_every);
  }
  if (e != hipSuccess || *status != SSO_OK) return e;
  return pcg_correct(m, pat, K, Dinv, b, x, rtol, max_it, w, s, iters, status);
}

// FP64 iterative refinement after a converged PCG: while the true residual b - K x is above
// rtol |b| (the recursive residual drifted below it), solve K d = r for the missing reduction
// and set x += d.  Stops when the target is met, refinement stalls (status SSO_ENOTCONV) or
// after 3 steps.
hipError_t pcg_correct(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                       const double* b, double* x, double rtol, int max_it, PcgWork& w,
                       hipStream_t s, int* iters, int* status) {
  hipError_t e;
  double* scal = part_once(w) + 2 * (size_t)partial_stride(w);
  double prev = -1.0;
  for (int step = 0; step <= 3; ++step) {
    if ((e = launch_true_residual(m, pat, K, x, b, w.r, w, scal, s)) != hipSuccess) return e;
    double h[2];
    if ((e = hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const double rn = std::sqrt(h[0]), bn = std::sqrt(h[1]);
    if (!(rn > rtol * bn)) {
      *status = std::isfinite(rn) ? SSO_OK : SSO_EBREAKDOWN;
      return hipSuccess;
    }
    if (step == 3 || (prev >= 0.0 && rn > 0.5 * prev) || *iters >= max_it) {
      *status = SSO_ENOTCONV;
      return hipSuccess;
    }
    prev = rn;
    double tol_k = 0.5 * rtol * bn / rn;
    if (tol_k > 0.5) tol_k = 0.5;
    int it = 0, st = SSO_OK;
    // correction d in w.Ap-free storage: solve into the second direction buffer's partner x2
    if ((e = pcg_run<double>(m, pat, K, Dinv, w.r, w.xc, w.rc, w.z, w.p, w.Ap, tol_k,
                             max_it - *iters, w, s, &it, &st, 0)) != hipSuccess)
      return e;
    *iters += it;
    if ((e = launch_axpy(1.0, w.xc, x, w.n_dof, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Mixed precision: FP64 flexible conjugate gradients (Notay's FCG with one stored direction)
// whose preconditioner is an FP32 PCG solve (FP32 K, vectors, SpMV and workgroup
// accumulation).  Each outer step: inner solve K d = r / |r| in FP32 to the tolerance still
// missing (factor 2 of margin, clamped to [inner_rtol, 0.5]) or inner_max_it iterations;
// z = |r| d; p = z - beta p_prev, q = K p in FP64; x += alpha p, r -= alpha q.  Because alpha
// and beta come from FP64 products with the FP64 K, a crude inner solve (a few iterations, or
// an FP32 operator too far from K for plain refinement) still makes progress.  When the
// recursive residual meets the target, the true residual is recomputed; if it misses, the
// iteration restarts from it (at most twice).
// Kept as a step machine, so that single solves and multi-problem launches share it:
// mixed_begin starts the first inner solve, mixed_inner_done takes the stopped inner solve
// through the outer step and starts the next one (or stops: ms.done, ms.status).
static constexpr int FCG_RESTARTS = 2;

static int64_t fcg_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return g > 1024 ? 1024 : (g < 1 ? 1 : g);
}

static double* fcg_scalars(PcgWork& w) { return part_once(w) + 2 * (size_t)partial_stride(w); }

// Read sc[0..4] back (synchronises the stream).
static hipError_t fcg_read(PcgWork& w, hipStream_t s, double h[5]) {
  hipError_t e = hipMemcpyAsync(h, fcg_scalars(w), 5 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// With the residual norm rn of r (w.r), stop or start the next inner solve.
static hipError_t mixed_next(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                             const float* Dinv32, const float* B32, const double* b, double* x,
                             const MixedParams& mp, PcgWork& w, hipStream_t s, MixedState& ms,
                             double rn) {
  hipError_t e;
  const int64_t n = w.n_dof;
  ms.done = true;
  if (!std::isfinite(rn)) {
    ms.status = SSO_EBREAKDOWN;
    return hipSuccess;
  }
  if (rn <= mp.rtol * ms.bn) {
    if (ms.outer == 0) {
      ms.status = SSO_OK;
      return hipSuccess;
    }
    double* sc = fcg_scalars(w);
    if ((e = launch_true_residual(m, pat, K, x, b, w.r, w, sc, s)) != hipSuccess) return e;
    double h[5];
    if ((e = fcg_read(w, s, h)) != hipSuccess) return e;
    const double rt = std::sqrt(h[0]);
    if (rt <= mp.rtol * ms.bn) {
      ms.status = SSO_OK;
      return hipSuccess;
    }
    if (ms.restarts == FCG_RESTARTS || !std::isfinite(rt)) {
      ms.status = SSO_ENOTCONV;   // the recursive residual drifted from the true one
      return hipSuccess;
    }
    ++ms.restarts;
    ms.k = 0;
    rn = rt;
  }
  const int left = mp.max_it - ms.iters;
  if (ms.outer == mp.refine_steps || left <= 0) {
    ms.status = SSO_ENOTCONV;   // outer limit reached or iterations used up
    return hipSuccess;
  }
  ms.done = false;
  ms.rn = rn;
  hipLaunchKernelGGL(k_scale_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, w.r, 1.0 / rn,
                     w.b32);
  double tol_k = 0.5 * mp.rtol * ms.bn / rn;
  if (tol_k < mp.inner_rtol) tol_k = mp.inner_rtol;
  if (tol_k > 0.5) tol_k = 0.5;
  const int cap = (mp.inner_max_it > 0 && mp.inner_max_it < left) ? mp.inner_max_it : left;
  if (B32) {
    const FusedBuffers<float> v{w.x32, w.p32[0], {w.r32, w.z32}, {w.p32[1], w.Ap32},
                                {w.fw32[0], w.fw32[1]}};
    ms.fdesc = fused_desc(m, pat, B32, Dinv32, (const float*)w.b32, v, w);
    FusedDesc<float>* dd = nullptr;
    if ((e = fused_start(ms.fdesc, tol_k, cap, w, s, &dd)) != hipSuccess) return e;
  } else {
    if ((e = pcg_start<float>(m, pat, K32, Dinv32, w.b32, w.x32, w.r32, w.z32, w.p32, w.Ap32,
                              tol_k, cap, w, s, &ms.sdesc)) != hipSuccess)
      return e;
  }
  w.h_st->done = 0;
  return hipSuccess;
}

// The outer step after an inner solve stopped.
static hipError_t mixed_inner_done(const Mesh& m, const Pattern& pat, const double* K,
                                   const float* K32, const float* Dinv32, const float* B32,
                                   const double* b, double* x, const MixedParams& mp, PcgWork& w,
                                   hipStream_t s, MixedState& ms) {
  const int it = w.h_st->it;
  const int st = w.h_st->done ? w.h_st->status : SSO_ENOTCONV;
  ms.iters += it;
  ++ms.outer;
  if (st == SSO_EBREAKDOWN && it == 0) {
    ms.done = true;
    ms.status = SSO_EBREAKDOWN;
    return hipSuccess;
  }
  const int64_t n = w.n_dof;
  const int g = (int)fcg_grid(n);
  double* sc = fcg_scalars(w);
  double* part = part_once(w);
  double* p_prev = w.p[ms.k & 1];
  double* p_new = w.p[(ms.k + 1) & 1];
  hipLaunchKernelGGL(k_fcg_z, dim3(g), dim3(256), 0, s, n, ms.rn, w.x32, w.Ap, w.z,
                     ms.k > 0 ? 1 : 0, part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, part, g, 1, sc + 2);
  hipLaunchKernelGGL(k_fcg_direction, dim3(w.n_wg), dim3(MAX_TPB), 0, s, m.n_nodes,
                     pat.brow_ptr, pat.bcol, K, w.z, p_prev, w.r, sc, ms.k == 0 ? 1 : 0, p_new,
                     w.Ap, part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, part, w.n_wg, 2, sc + 3);
  hipLaunchKernelGGL(k_fcg_update, dim3(g), dim3(256), 0, s, n, sc, p_new, w.Ap, x, w.r, part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, part, g, 1, sc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double h[5];
  if ((e = fcg_read(w, s, h)) != hipSuccess) return e;
  if (!(h[3] > 0.0)) {
    // p^T K p <= 0: zero direction (the inner solve returned nothing) or not finite
    ms.done = true;
    ms.status = std::isfinite(h[3]) ? SSO_ENOTCONV : SSO_EBREAKDOWN;
    return hipSuccess;
  }
  ++ms.k;
  return mixed_next(m, pat, K, K32, Dinv32, B32, b, x, mp, w, s, ms, std::sqrt(h[0]));
}

hipError_t mixed_begin(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                       const float* Dinv32, const float* B32, const double* b, double* x,
                       const MixedParams& mp, PcgWork& w, hipStream_t s, MixedState& ms) {
  hipError_t e;
  if ((e = pcg_alloc_mixed(w, s)) != hipSuccess) return e;
  if (B32 && (e = fused_alloc(w, true, s)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(x, 0, sizeof(double) * (size_t)w.n_dof, s)) != hipSuccess) return e;
  ms = MixedState();
  // r = b - K 0 = b, and |b|
  if ((e = launch_true_residual(m, pat, K, x, b, w.r, w, fcg_scalars(w), s)) != hipSuccess)
    return e;
  double h[5];
  if ((e = fcg_read(w, s, h)) != hipSuccess) return e;
  ms.bn = std::sqrt(h[1]);
  return mixed_next(m, pat, K, K32, Dinv32, B32, b, x, mp, w, s, ms, std::sqrt(h[0]));
}

hipError_t mixed_step(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                      const float* Dinv32, const float* B32, const double* b, double* x,
                      const MixedParams& mp, PcgWork& w, hipStream_t s, MixedState& ms) {
  if (ms.done || !w.h_st->done) return hipSuccess;
  return mixed_inner_done(m, pat, K, K32, Dinv32, B32, b, x, mp, w, s, ms);
}

hipError_t pcg_solve_mixed(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                           const float* Dinv32, const float* B32, const double* b, double* x,
                           const MixedParams& mp, PcgWork& w, hipStream_t s, int* iters,
                           int* status, int* outer, int profile_every) {
  w.prof_us = 0.0;
  w.prof_n = 0;
  MixedState ms;
  hipError_t e = mixed_begin(m, pat, K, K32, Dinv32, B32, b, x, mp, w, s, ms);
  while (e == hipSuccess && !ms.done) {
    int it = 0, st = SSO_OK;
    const int nwg = B32 ? w.n_wg_f : w.n_wg;
    const int left = mp.max_it - ms.iters;
    // the inner solve's own limit (set on the device by mixed_next)
    const int cap = (mp.inner_max_it > 0 && mp.inner_max_it < left) ? mp.inner_max_it : left;
    if (B32) {
      const FusedDesc<float> hd = ms.fdesc;
      int k = 0;
      auto launch = [&](hipEvent_t* e0, hipEvent_t* e1) {
        if (e0) (void)hipEventRecord(*e0, s);
        launch_iter1(hd, nwg, k, s);
        if (e1) (void)hipEventRecord(*e1, s);
        ++k;
      };
      e = run_polled(w, s, cap, profile_every, FUSED_SPAN, launch, &it, &st);
    } else {
      const PcgDesc<float>* dd = reinterpret_cast<const PcgDesc<float>*>(w.desc32);
      // the single-problem kernels with their first group's fields preloaded (forced mixed
      // precision: 300 x 300 shell at 1e-10 575.4-575.5 against 576.6-578.0 ms, 250 x 250 at
      // 1e-8 259.0-260.7 against 262.5-263.4 ms)
      auto launch = [&](hipEvent_t* e0, hipEvent_t* e1) {
        if (e0) (void)hipEventRecord(*e0, s);
        const PcgDesc<float>& hd = ms.sdesc;
        hipLaunchKernelGGL((k_spmv_dir_single<float, false>), dim3(nwg), dim3(MAX_TPB), 0, s,
                           hd.brow_ptr, hd.st, (const double*)hd.pb, hd.n_nodes, hd.n_wg, dd);
        hipLaunchKernelGGL(k_update_single<float>, dim3(update_wg(nwg, m.n_nodes)),
                           dim3(MAX_TPB), 0, s, hd.n_nodes, hd.n_wg, (const float*)hd.Ap, hd.r,
                           hd.p[0], hd.p[1], (const double*)hd.pa, hd.st, dd);
        if (e1) (void)hipEventRecord(*e1, s);
      };
      e = run_polled(w, s, cap, profile_every, cap >= STD_SPAN ? STD_SPAN : 1, launch, &it, &st);
    }
    if (e == hipSuccess) e = mixed_inner_done(m, pat, K, K32, Dinv32, B32, b, x, mp, w, s, ms);
  }
  *iters = ms.iters;
  *status = ms.status;
  *outer = ms.outer;
  return e;
}

hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(nblk(n, 256)), dim3(256), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_f32, dim3(nblk(n, 256)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}

hipError_t launch_dot(const double* a, const double* b, int64_t n, PcgWork& w, double* d_out,
                      hipStream_t s) {
  int nwg = (int)((n + 255) / 256);
  if (nwg > 1024) nwg = 1024;
  if (nwg < 1) nwg = 1;
  double* part = part_once(w);
  hipLaunchKernelGGL(k_dot, dim3(nwg), dim3(256), 0, s, n, a, b, part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, part, nwg, 1, d_out);
  return hipGetLastError();
}

hipError_t launch_true_residual(const Mesh& m, const Pattern& pat, const double* K,
                                const double* x, const double* b, double* r, PcgWork& w,
                                double* d_out, hipStream_t s) {
  double* part = part_once(w);
  hipLaunchKernelGGL(k_residual, dim3(w.n_wg), dim3(MAX_TPB), 0, s, m.n_nodes, pat.brow_ptr,
                     pat.bcol, K, x, b, r, part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, part, w.n_wg, 2, d_out);
  return hipGetLastError();
}

double fused_bytes_per_iteration(int64_t n_nodes, int64_t n_blocks, bool mixed) {
  const double n_dof = 6.0 * (double)n_nodes, v = mixed ? 4.0 : 8.0;
  // B values + block columns + row pointers; r, w, s gathered; p, x read; Dinv (21 per node,
  // 3.5 per DOF); p, x, s, r, w written
  return (36.0 * v + 4.0) * n_blocks + 4.0 * (n_nodes + 1) + (3 + 2 + 3.5 + 5) * v * n_dof;
}

bool pcg_sym_products(int64_t n_blocks, bool mixed) {
  return !mixed && 36.0 * 8.0 * (double)n_blocks >= SYM_PRODUCT_MIN_K_BYTES;
}

double spmv_bytes_per_launch(int64_t n_nodes, int64_t n_blocks, bool mixed, bool sym) {
  const double fb = mixed ? 4.0 : 8.0;
  const double tail = 4.0 * (n_nodes + 1) + 4.0 * fb * 6.0 * n_nodes;
  // upper triangle: the diagonal and half the off-diagonal blocks, (column, value slot) pairs
  if (sym) return 36.0 * fb * 0.5 * (double)(n_blocks + n_nodes) + 8.0 * n_blocks + tail;
  return 36.0 * fb * n_blocks + 4.0 * n_blocks + tail;
}

double pcg_bytes_per_iteration(int64_t n_nodes, int64_t n_blocks, bool mixed, bool sym) {
  const double fb = mixed ? 4.0 : 8.0;
  const double n_dof = 6.0 * (double)n_nodes;
  // spmv: K values (the upper triangle: sym) + block columns + row pointers; z, p_old read;
  // p_new, Ap written
  double spmv = spmv_bytes_per_launch(n_nodes, n_blocks, mixed, sym);
  // update: x, p, Ap, r read, Dinv (21 per node, 3.5 per DOF); x, r, z written
  double upd = 4.0 * fb * n_dof + 3.5 * fb * n_dof + 3.0 * fb * n_dof;
  return spmv + upd;
}

}  // namespace sso
