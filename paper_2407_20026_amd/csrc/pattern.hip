// Sparse pattern of K and the scatter permutation, built once per topology.
//
// Sec. 2.2.1: every element has an index map from its local matrix entries to rows and columns
// of the global K, and K is stored sparse.  Here the map is built at the granularity of 6x6 node
// blocks: each element contributes one block per ordered pair of its nodes ("block
// contributions": 4 per member, 16 per quad, id j = 4 e + 2 la + lb for members and
// 4 nb + 16 e + 4 la + lb for quads).  Contributions are bucketed by block row with integer
// atomics, then each row is sorted by the full key (column, id).  Because the key is unique,
// the result does not depend on the order in which the atomics were served: the permutation is
// the stable sort of the contribution list by (row, column), bit for bit.  The scalar CSR view
// (row = 6 I + a, column = 6 J + b) and its permutation follow in closed form from the block
// data because all 36 entries of a block contribution share the block's rank.
#include "sso_internal.h"

namespace sso {
namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(int64_t n, int tpb = TPB) {
  return (unsigned)((n + tpb - 1) / tpb);
}

__device__ inline void node_pair(const Mesh& m, const BlockRef& r, int& I, int& J) {
  if (!r.quad) {
    I = m.beam_nodes[2 * (int64_t)r.e + r.la];
    J = m.beam_nodes[2 * (int64_t)r.e + r.lb];
  } else {
    I = m.quad_nodes[4 * (int64_t)r.e + r.la];
    J = m.quad_nodes[4 * (int64_t)r.e + r.lb];
  }
}

__global__ void k_block_count(Mesh m, int64_t n_bcoo, int32_t* cnt, unsigned* err) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n_bcoo) return;
  BlockRef r = decode_block(j, m.n_beams);
  int I, J;
  node_pair(m, r, I, J);
  if (I < 0 || I >= m.n_nodes || J < 0 || J >= m.n_nodes) {
    atomicOr(err, ERR_INDEX);
    return;
  }
  if (r.la != r.lb && I == J) {
    atomicOr(err, ERR_REPEAT);
    return;
  }
  atomicAdd(&cnt[I], 1);
}

__global__ void k_block_place(Mesh m, int64_t n_bcoo, const int32_t* estart, int32_t* fill,
                              uint64_t* keys) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n_bcoo) return;
  BlockRef r = decode_block(j, m.n_beams);
  int I, J;
  node_pair(m, r, I, J);
  int pos = estart[I] + atomicAdd(&fill[I], 1);
  keys[pos] = ((uint64_t)(uint32_t)J << 32) | (uint64_t)(uint32_t)j;
}

// Insertion sort of each row's keys (rows hold a handful of entries: 16 for an interior node
// of a quad grid), then the number of distinct block columns.
__global__ void k_row_sort(int n_nodes, const int32_t* estart, uint64_t* keys, int32_t* ucnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  int b = estart[I], e = estart[I + 1];
  for (int i = b + 1; i < e; ++i) {
    uint64_t k = keys[i];
    int q = i - 1;
    while (q >= b && keys[q] > k) {
      keys[q + 1] = keys[q];
      --q;
    }
    keys[q + 1] = k;
  }
  int u = 0;
  uint32_t prev = 0xffffffffu;
  for (int i = b; i < e; ++i) {
    uint32_t J = (uint32_t)(keys[i] >> 32);
    if (J != prev) ++u;
    prev = J;
  }
  ucnt[I] = (e > b) ? u : 1;   // an isolated node keeps its (empty) diagonal block
}

__global__ void k_emit(int n_nodes, const int32_t* estart, const uint64_t* keys,
                       const int32_t* brow_ptr, int32_t* bcol, int32_t* bseg, int32_t* bperm,
                       int32_t* bslot, int32_t* bdiag, int32_t* bsrow) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n_nodes) return;
  int b = estart[I], e = estart[I + 1];
  int s = brow_ptr[I] - 1;
  if (e == b) {
    s = brow_ptr[I];
    bcol[s] = I;
    bseg[s] = b;
    bdiag[I] = s;
    bsrow[s] = I;
    return;
  }
  uint32_t prev = 0xffffffffu;
  for (int i = b; i < e; ++i) {
    uint32_t J = (uint32_t)(keys[i] >> 32);
    if (J != prev) {
      ++s;
      bcol[s] = (int32_t)J;
      bseg[s] = i;
      bsrow[s] = I;
      if ((int)J == I) bdiag[I] = s;
    }
    prev = J;
    bperm[i] = (int32_t)(uint32_t)(keys[i] & 0xffffffffu);
    bslot[i] = s;
  }
}

// (column, value slot) of each slot: a block (I, J) with J < I takes the values of block (J, I)
// (an element couples its nodes both ways, so that block exists; found by bisection in row J's
// sorted columns), any other block its own.
__global__ void k_sym_slots(int64_t n_blocks, const int32_t* brow_ptr, const int32_t* bcol,
                            const int32_t* bsrow, int32_t* bsym) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n_blocks) return;
  const int I = bsrow[s], J = bcol[s];
  int m = (int)s;
  if (J < I) {
    int lo = brow_ptr[J], hi = brow_ptr[J + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (bcol[mid] < I)
        lo = mid + 1;
      else
        hi = mid;
    }
    m = lo;
  }
  bsym[2 * s] = J;
  bsym[2 * s + 1] = m;
}

// ---- exclusive scan of int32 counts (n entries) into out[0..n], out[n] = total -------------

constexpr int SCAN_TPB = 256;
constexpr int SCAN_PER = 8;
constexpr int SCAN_TILE = SCAN_TPB * SCAN_PER;

__device__ inline int block_exclusive_scan(int v, int* lds, int& total) {
  // Hillis-Steele over one workgroup (fixed order: integer, exact)
  int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_TPB; off <<= 1) {
    int add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  total = lds[SCAN_TPB - 1];
  int incl = lds[t];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_tile_sums(const int32_t* in, int64_t n, int32_t* tile_sums) {
  __shared__ int lds[SCAN_TPB];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
  int s = 0;
  for (int k = 0; k < SCAN_PER; ++k)
    if (base + k < n) s += in[base + k];
  int total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_tile_offsets(int32_t* tile_sums, int n_tiles) {
  __shared__ int lds[SCAN_TPB];
  int carry = 0;
  for (int base = 0; base < n_tiles; base += SCAN_TPB) {
    int i = base + threadIdx.x;
    int v = (i < n_tiles) ? tile_sums[i] : 0;
    int total;
    int ex = block_exclusive_scan(v, lds, total);
    if (i < n_tiles) tile_sums[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sums[n_tiles] = carry;
}

__global__ void k_scan_apply(const int32_t* in, int64_t n, const int32_t* tile_offsets,
                             int32_t* out) {
  __shared__ int lds[SCAN_TPB];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
  int v[SCAN_PER];
  int s = 0;
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int ex = block_exclusive_scan(s, lds, total) + tile_offsets[blockIdx.x];
  for (int k = 0; k < SCAN_PER; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_offsets[gridDim.x];
}

hipError_t exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp,
                          hipStream_t s) {
  int n_tiles = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
  if (n_tiles == 0) n_tiles = 1;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(n_tiles), dim3(SCAN_TPB), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(SCAN_TPB), 0, s, tmp, n_tiles);
  hipLaunchKernelGGL(k_scan_apply, dim3(n_tiles), dim3(SCAN_TPB), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

// ---- scalar CSR view ----------------------------------------------------------------------

__global__ void k_scalar_rows(int n_nodes, int64_t n_blocks, int64_t n_coo,
                              const int32_t* brow_ptr, const int32_t* bcol, const int32_t* bseg,
                              const int32_t* estart, int32_t* row_ptr, int32_t* col,
                              int32_t* seg) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= 6 * (int64_t)n_nodes) return;
  int I = (int)(t / 6), a = (int)(t % 6);
  int rb = brow_ptr[I], re = brow_ptr[I + 1];
  int nbc = re - rb;
  int es = estart[I], nent = estart[I + 1] - es;
  int64_t rp = 36 * (int64_t)rb + 6 * (int64_t)a * nbc;
  row_ptr[t] = (int32_t)rp;
  for (int k = 0; k < nbc; ++k) {
    int sl = rb + k;
    int cnt = bseg[sl + 1] - bseg[sl];
    int64_t first = 36 * (int64_t)es + 6 * (int64_t)a * nent + 6 * (int64_t)(bseg[sl] - es);
    for (int b = 0; b < 6; ++b) {
      col[rp + 6 * k + b] = 6 * bcol[sl] + b;
      seg[rp + 6 * k + b] = (int32_t)(first + (int64_t)b * cnt);
    }
  }
  if (t == 0) {
    row_ptr[6 * (int64_t)n_nodes] = (int32_t)(36 * n_blocks);
    seg[36 * n_blocks] = (int32_t)n_coo;
  }
}

__global__ void k_scalar_perm(Mesh m, int64_t n_bcoo, const int32_t* bperm, const int32_t* bslot,
                              const int32_t* bseg, const int32_t* estart, int32_t* perm) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n_bcoo) return;
  int j = bperm[p];
  int sl = bslot[p];
  BlockRef r = decode_block(j, m.n_beams);
  int I, J;
  node_pair(m, r, I, J);
  int es = estart[I], nent = estart[I + 1] - es;
  int cnt = bseg[sl + 1] - bseg[sl];
  int rank = (int)(p - bseg[sl]);
  for (int a = 0; a < 6; ++a) {
    int64_t base = 36 * (int64_t)es + 6 * (int64_t)a * nent + 6 * (int64_t)(bseg[sl] - es) + rank;
    for (int b = 0; b < 6; ++b)
      perm[base + (int64_t)b * cnt] = (int32_t)coo_index(r, a, b, m.n_beams);
  }
}

}  // namespace

#define SSO_TRY(x)                 \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Largest block count of a row (one workgroup, fixed order).
__global__ void __launch_bounds__(256) k_max_row(int n_nodes, const int32_t* brow_ptr,
                                                 int32_t* out) {
  __shared__ int32_t sm[256];
  int32_t mx = 0;
  for (int i = threadIdx.x; i < n_nodes; i += blockDim.x) {
    const int32_t c = brow_ptr[i + 1] - brow_ptr[i];
    mx = c > mx ? c : mx;
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h && sm[threadIdx.x + h] > sm[threadIdx.x])
      sm[threadIdx.x] = sm[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// Padded block columns: slot u of row I is the row's u-th block column, or I past its count.
__global__ void k_ell_cols(int n_nodes, int w, const int32_t* brow_ptr, const int32_t* bcol,
                           int32_t* bcol_ell) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_nodes * w) return;
  const int I = (int)(e / w), u = (int)(e - (int64_t)I * w);
  const int rb = brow_ptr[I], cnt = brow_ptr[I + 1] - rb;
  bcol_ell[e] = u < cnt ? bcol[rb + u] : I;
}

hipError_t build_pattern(const Mesh& m, Pattern& pat, unsigned* d_err, hipStream_t s,
                         unsigned* h_err) {
  const int n = m.n_nodes;
  pat.n_bcoo = 4 * (int64_t)m.n_beams + 16 * (int64_t)m.n_quads;
  int32_t *cnt = nullptr, *fill = nullptr, *tmp = nullptr, *ucnt = nullptr;
  uint64_t* keys = nullptr;
  int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE + 2;
  int64_t nk = pat.n_bcoo > 0 ? pat.n_bcoo : 1;
  // the build's own scratch: one arena, freed on every way out of this function
  Arena scratch;
  struct Release {
    Arena& a;
    hipStream_t s;
    ~Release() { arena_free(a, s); }
  } release{scratch, s};
  {
    AllocScope sc(nullptr, &scratch);
    SSO_TRY(dev_alloc(&cnt, (n + 1), s));
    SSO_TRY(dev_alloc(&fill, (n + 1), s));
    SSO_TRY(dev_alloc(&ucnt, (n + 1), s));
    SSO_TRY(dev_alloc(&tmp, nt, s));
    SSO_TRY(dev_alloc(&keys, nk, s));
  }
  SSO_TRY(dev_alloc(&pat.estart, (n + 1), s));
  SSO_TRY(dev_alloc(&pat.brow_ptr, (n + 1), s));
  SSO_TRY(dev_alloc(&pat.bperm, nk, s));
  SSO_TRY(dev_alloc(&pat.bslot, nk, s));
  SSO_TRY(dev_alloc(&pat.bdiag, n, s));
  SSO_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), s));
  SSO_TRY(hipMemsetAsync(fill, 0, sizeof(int32_t) * (n + 1), s));
  if (pat.n_bcoo)
    hipLaunchKernelGGL(k_block_count, dim3(blocks_for(pat.n_bcoo)), dim3(TPB), 0, s, m,
                       pat.n_bcoo, cnt, d_err);
  SSO_TRY(hipGetLastError());
  SSO_TRY(hipMemcpyAsync(h_err, d_err, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  SSO_TRY(hipStreamSynchronize(s));
  if (*h_err) return hipSuccess;   // caller reports SSO_EINVAL
  SSO_TRY(exclusive_scan(cnt, n, pat.estart, tmp, s));
  if (pat.n_bcoo)
    hipLaunchKernelGGL(k_block_place, dim3(blocks_for(pat.n_bcoo)), dim3(TPB), 0, s, m,
                       pat.n_bcoo, pat.estart, fill, keys);
  hipLaunchKernelGGL(k_row_sort, dim3(blocks_for(n)), dim3(TPB), 0, s, n, pat.estart, keys,
                     ucnt);
  SSO_TRY(hipGetLastError());
  SSO_TRY(exclusive_scan(ucnt, n, pat.brow_ptr, tmp, s));
  int32_t nblk = 0;
  SSO_TRY(hipMemcpyAsync(&nblk, pat.brow_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SSO_TRY(hipStreamSynchronize(s));
  pat.n_blocks = nblk;
  SSO_TRY(dev_alloc(&pat.bcol, nblk, s));
  SSO_TRY(dev_alloc(&pat.bseg, (nblk + 1), s));
  SSO_TRY(dev_alloc(&pat.bsrow, nblk, s));
  hipLaunchKernelGGL(k_emit, dim3(blocks_for(n)), dim3(TPB), 0, s, n, pat.estart, keys,
                     pat.brow_ptr, pat.bcol, pat.bseg, pat.bperm, pat.bslot, pat.bdiag, pat.bsrow);
  SSO_TRY(hipGetLastError());
  int32_t last = (int32_t)pat.n_bcoo;
  SSO_TRY(hipMemcpyAsync(pat.bseg + nblk, &last, sizeof(int32_t), hipMemcpyHostToDevice, s));
  SSO_TRY(dev_alloc(&pat.bsym, 2 * (int64_t)nblk, s));
  hipLaunchKernelGGL(k_sym_slots, dim3(blocks_for(nblk)), dim3(TPB), 0, s, (int64_t)nblk,
                     pat.brow_ptr, pat.bcol, pat.bsrow, pat.bsym);
  SSO_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_max_row, dim3(1), dim3(256), 0, s, n, pat.brow_ptr, tmp);
  SSO_TRY(hipGetLastError());
  int32_t max_row = 0;
  SSO_TRY(hipMemcpyAsync(&max_row, tmp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SSO_TRY(hipStreamSynchronize(s));
  pat.ell_w = ell_width(max_row);
  if (pat.ell_w) {
    const int64_t ne = (int64_t)n * pat.ell_w;
    SSO_TRY(dev_alloc(&pat.bcol_ell, ne, s));
    hipLaunchKernelGGL(k_ell_cols, dim3(blocks_for(ne)), dim3(TPB), 0, s, n, pat.ell_w,
                       pat.brow_ptr, pat.bcol, pat.bcol_ell);
    SSO_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t build_scalar_view(const Mesh& m, const Pattern& pat, int32_t* row_ptr, int32_t* col,
                             int32_t* perm, int32_t* seg, hipStream_t s) {
  int64_t n_coo = 144 * (int64_t)m.n_beams + 576 * (int64_t)m.n_quads;
  hipLaunchKernelGGL(k_scalar_rows, dim3(blocks_for(6 * (int64_t)m.n_nodes)), dim3(TPB), 0, s,
                     m.n_nodes, pat.n_blocks, n_coo, pat.brow_ptr, pat.bcol, pat.bseg, pat.estart,
                     row_ptr, col, seg);
  if (pat.n_bcoo)
    hipLaunchKernelGGL(k_scalar_perm, dim3(blocks_for(pat.n_bcoo)), dim3(TPB), 0, s, m,
                       pat.n_bcoo, pat.bperm, pat.bslot, pat.bseg, pat.estart, perm);
  return hipGetLastError();
}

void free_pattern(Pattern& pat, hipStream_t s) {
  for (void* q : {(void*)pat.brow_ptr, (void*)pat.bcol, (void*)pat.bseg, (void*)pat.bperm,
                  (void*)pat.bslot, (void*)pat.bdiag, (void*)pat.estart, (void*)pat.bsrow,
                  (void*)pat.bcol_ell, (void*)pat.bsym})
    dev_release(q, &pat.mem, s);
  arena_free(pat.mem, s);
  pat = Pattern();
}

}  // namespace sso
