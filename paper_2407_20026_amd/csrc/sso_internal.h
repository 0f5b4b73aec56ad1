// Internal declarations shared by the translation units of libhipsso.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <utility>
#include <vector>

#include "hipsso.h"

namespace sso {

// Error bits raised by kernels (OR-ed into a device word; read back by the host).
enum : unsigned {
  ERR_INDEX = 1u << 0,       // node index out of range
  ERR_REPEAT = 1u << 1,      // element repeats a node
  ERR_BEAM = 1u << 2,        // zero-length member or non-positive section property
  ERR_QUAD = 1u << 3,        // det J <= 0, zero area, bad t/E/nu, kx/ky != 1
  ERR_DIAG = 1u << 4,        // diagonal 6x6 block not positive definite
  ERR_TOPO = 1u << 5,        // connectivity differs from the problem whose pattern is shared
};

// PCG scalar state record in device memory (written by workgroup 0 of the PCG kernels, polled
// by the host between chunks of iterations).
struct PcgState {
  double rzs[2];   // r_j^T z_j by iteration parity
  double alphas[2];  // alpha_j by iteration parity (single-reduction variant)
  double rr;       // r^T r of the last finished iteration
  double ff;       // ||rhs||^2
  double rtol2;    // rtol^2
  int it;          // iterations done
  int done;        // 1: stop (converged, breakdown, or limit)
  int status;      // SSO_OK, SSO_ENOTCONV, SSO_EBREAKDOWN
  int max_it;
  int jn;          // index of the next iteration (written by the update kernel)
  int jc;          // index of the iteration in flight (written by the SpMV kernel)
};

// One problem of a PCG launch: operands, work vectors, partial sums, state record, and its
// range of workgroups in the launch.
template <class T>
struct PcgDesc {
  const int32_t* brow_ptr;
  const int32_t* bcol;
  const int32_t* bsym;      // (column, value slot) of each block slot
  const T* K;
  const T* Dinv;
  const T* b;
  T* x;
  T* r;
  T* z;
  T* p[2];
  T* Ap;
  double* pa;
  double* pb;
  PcgState* st;
  int n_nodes, n_wg, wg_base;
  int stream_stores;   // 1: the vectors an iteration writes go out as streaming stores
  int64_t n_blocks;    // blocks of K
};

// One problem of a single-reduction PCG launch (one kernel and one reduction per iteration).
template <class T>
struct FusedDesc {
  const int32_t* brow_ptr;
  const int32_t* bcol;
  const int32_t* bcol_ell;   // padded block-row columns (ell_w > 0)
  const T* B;       // K times the block-Jacobi inverse: padded layout (ell_w > 0) or K's
  const T* Dinv;
  const T* b;
  T* x;
  T* p;
  T* r[2];
  T* w[2];
  T* s[2];
  double* pp[2];
  int32_t* jw;      // per-workgroup iteration counters
  PcgState* st;
  int n_nodes, n_wg, wg_base, ell_w;
  double rtol2;     // squared relative tolerance and iteration limit of the running solve
  int max_it;       //   (set when it starts; read by the single-problem iteration)
};

// Memory that lives as long as its owner (a problem, a block pattern) is carved from a few
// chunks of the pool and freed with them when the owner ends: a stream-ordered free costs about
// 20 us of host time, and a problem has some 45 buffers.  A buffer above ARENA_CHUNK / 4 gets a
// chunk of its own; smaller ones share chunks of ARENA_CHUNK bytes, and a chunk is left only when
// less than ARENA_CHUNK / 4 of it is free, so every chunk but the last is at least 3/4 used.
struct Arena {
  std::vector<std::pair<char*, size_t>> chunks;   // base, size
  char* cur = nullptr;
  size_t left = 0;
};
constexpr size_t ARENA_CHUNK = (size_t)2 << 20;
constexpr size_t ARENA_ALIGN = 256;

// Block-level pattern (6x6 blocks, one block row per node).
struct Pattern {
  int64_t n_bcoo = 0;       // block contributions: 4 per beam, 16 per quad
  int64_t n_blocks = 0;     // 6x6 blocks of K
  int32_t* brow_ptr = nullptr;  // [n_nodes + 1]
  int32_t* bcol = nullptr;      // [n_blocks]
  int32_t* bseg = nullptr;      // [n_blocks + 1] segment of each block slot in bperm
  int32_t* bperm = nullptr;     // [n_bcoo] block contribution ids sorted by (row, col, id)
  int32_t* bslot = nullptr;     // [n_bcoo] slot of each sorted position
  int32_t* bdiag = nullptr;     // [n_nodes] slot of the diagonal block of each row
  int32_t* bsrow = nullptr;     // [n_blocks] block row of each slot
  int32_t* estart = nullptr;    // [n_nodes + 1] first sorted position of each block row
  // [2 n_blocks] per slot s of block (I, J): J, then the slot whose values the block takes
  // in the symmetric products (s itself for J >= I; the slot of (J, I) for J < I)
  int32_t* bsym = nullptr;
  // Padded layout of the block rows (every row ell_w slots; 0 = not built: a row has more
  // than 12 blocks): bcol_ell[I * ell_w + u] = column of block u of row I for u below the
  // row's block count, I itself (with a zero block) beyond.
  int ell_w = 0;
  int32_t* bcol_ell = nullptr;  // [n_nodes * ell_w]
  Arena mem;                    // chunks holding the arrays above
};

// Slots per row of the padded block-row layout for a largest row of `max_blocks` blocks; wider
// rows keep the row pointers (a padded FP64 row of 16 slots does not fit the registers of the
// fused iteration, whose spills would cost more memory traffic than the kernel's own).
inline int ell_width(int max_blocks) {
  return max_blocks <= 6 ? 6 : max_blocks <= 9 ? 9 : max_blocks <= 12 ? 12 : 0;
}

// The block-Jacobi inverse of a node is symmetric (W^T W): stored packed, its upper triangle
// row by row (21 values per node), entry (a, b) at dinv_index(a, b).  The array is padded to
// whole groups of 64 nodes, so that the vector kernels can stage a group's 21 x 64 values with
// 16-byte loads without a bound test.
constexpr int DINV_PACKED = 21;
constexpr int DINV_GROUP = 64;
__host__ __device__ constexpr int dinv_index(int a, int b) {
  return a <= b ? a * (11 - a) / 2 + b : b * (11 - b) / 2 + a;
}
inline int64_t dinv_packed_len(int64_t n_nodes) {
  return DINV_PACKED * ((n_nodes + DINV_GROUP - 1) / DINV_GROUP) * DINV_GROUP;
}

struct Mesh {
  int32_t n_nodes = 0, n_beams = 0, n_quads = 0;
  double* xyz = nullptr;
  uint8_t* fixed = nullptr;
  double* f_nodal = nullptr;
  int32_t* beam_nodes = nullptr;
  double* beam_prop = nullptr;
  int32_t* quad_nodes = nullptr;
  double* quad_prop = nullptr;
  double* quad_scale = nullptr;   // always allocated when n_quads > 0 (1 when not given)
  double unit_weight = 0, surface_load = 0;
  double* u_presc = nullptr;      // [n_nodes][6] prescribed displacements, or null (all zero)
};

// Block contribution id j decoding: beams j = 4 e + 2 la + lb; quads j = 4 nb + 16 e + 4 la + lb.
struct BlockRef {
  int quad;   // 0 beam, 1 quad
  int e, la, lb;
};

__host__ __device__ inline BlockRef decode_block(int64_t j, int n_beams) {
  BlockRef r;
  int64_t nb4 = 4 * (int64_t)n_beams;
  if (j < nb4) {
    r.quad = 0;
    r.e = (int)(j >> 2);
    r.la = (int)((j >> 1) & 1);
    r.lb = (int)(j & 1);
  } else {
    int64_t q = j - nb4;
    r.quad = 1;
    r.e = (int)(q >> 4);
    r.la = (int)((q >> 2) & 3);
    r.lb = (int)(q & 3);
  }
  return r;
}

// Scalar index (into the element contribution list) of entry (ca, cb) of block contribution r.
__host__ __device__ inline int64_t coo_index(const BlockRef& r, int ca, int cb, int n_beams) {
  if (!r.quad) return 144 * (int64_t)r.e + 12 * (6 * r.la + ca) + 6 * r.lb + cb;
  return 144 * (int64_t)n_beams + 576 * (int64_t)r.e + 24 * (6 * r.la + ca) + 6 * r.lb + cb;
}

// Stream-ordered device memory from the library's pool on the stream's device (api.hip): no
// device-wide synchronisation, so problems that live on different streams keep overlapping
// while others are created or destroyed, and freed memory is reused without remapping.
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s);

// Carves `bytes` (rounded up to ARENA_ALIGN) on stream s; *held = bytes newly taken from the pool.
hipError_t arena_alloc(Arena& a, size_t bytes, hipStream_t s, void** out, int64_t* held);
bool arena_owns(const Arena& a, const void* p);
void arena_free(Arena& a, hipStream_t s);   // every chunk, stream-ordered on s

// While an entry point works on a problem, an AllocScope points this thread's allocations at
// the problem's arena and its byte count (sso_problem_bytes: the chunks held); the pattern build
// points them at the pattern's arena.  Outside a scope dev_alloc takes a buffer of its own from
// the pool (the multi-problem launch tables, which grow and shrink with the batch).
inline thread_local int64_t* alloc_counter = nullptr;
inline thread_local Arena* alloc_arena = nullptr;
struct AllocScope {
  int64_t* prev;
  Arena* prev_arena;
  AllocScope(int64_t* c, Arena* a) : prev(alloc_counter), prev_arena(alloc_arena) {
    alloc_counter = c;
    alloc_arena = a;
  }
  ~AllocScope() {
    alloc_counter = prev;
    alloc_arena = prev_arena;
  }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};

// A buffer of its own from the pool, never counted and never in an arena: for buffers freed
// with dev_free (the multi-problem launch tables and state arrays, owned by a batch).
template <class T>
inline hipError_t dev_alloc_scratch(T** p, int64_t n, hipStream_t s) {
  if (n <= 0) n = 1;
  return pool_alloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)n, s);
}
template <class T>
inline hipError_t dev_alloc(T** p, int64_t n, hipStream_t s) {
  if (n <= 0) n = 1;
  const size_t bytes = sizeof(T) * (size_t)n;
  if (alloc_arena) {
    int64_t held = 0;
    const hipError_t e = arena_alloc(*alloc_arena, bytes, s, reinterpret_cast<void**>(p), &held);
    if (e == hipSuccess && alloc_counter) *alloc_counter += held;
    return e;
  }
  const hipError_t e = dev_alloc_scratch(p, n, s);
  if (e == hipSuccess && alloc_counter) *alloc_counter += (int64_t)bytes;
  return e;
}
// Frees a buffer unless `owner` holds it in one of its chunks (freed with the owner).
inline void dev_release(void* p, const Arena* owner, hipStream_t s) {
  if (p && !(owner && arena_owns(*owner, p))) (void)hipFreeAsync(p, s);
}
inline void dev_free(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

// Host copies of a block pattern and the element connectivity, for check_pattern.
struct HostPattern {
  int n_nodes = 0, n_beams = 0, n_quads = 0, ell_w = 0;
  int64_t n_blocks = 0, n_bcoo = 0;
  const int32_t *brow_ptr = nullptr, *bcol = nullptr, *bseg = nullptr, *bperm = nullptr,
                *bslot = nullptr, *bdiag = nullptr, *bsrow = nullptr, *estart = nullptr,
                *bcol_ell = nullptr, *beam_nodes = nullptr, *quad_nodes = nullptr,
                *bsym = nullptr;
};
// validate.cpp: 0 when every invariant of the pattern holds, else the number of the first
// failed check (1-9) with a message in msg.
int check_pattern(const HostPattern& h, char* msg, size_t len);

// ---- launch helpers (each defined in its own translation unit) ----------------------------

// pattern.hip
hipError_t build_pattern(const Mesh& m, Pattern& pat, unsigned* d_err, hipStream_t s,
                         unsigned* h_err);
hipError_t build_scalar_view(const Mesh& m, const Pattern& pat, int32_t* row_ptr, int32_t* col,
                             int32_t* perm, int32_t* seg, hipStream_t s);
void free_pattern(Pattern& pat, hipStream_t s);

// elements.hip
hipError_t launch_element_stiffness(const Mesh& m, double* coo, double* qarea, unsigned* d_err,
                                    hipStream_t s);
hipError_t launch_adjoint_terms(const Mesh& m, const Pattern& pat, const double* u,
                                const double* lam, double c_lam, double c_u, double* gbeam,
                                double* gquad, hipStream_t s);
// Size optimisation objective pieces and the sensitivity hat filter (extras.hip, elements.hip).
hipError_t launch_volume_terms(const Mesh& m, double t_min, double* gw, double* w,
                               hipStream_t s);
hipError_t launch_size_terms(const Mesh& m, const double* u, double u_max, const double* w,
                             double* dcdu, double* partials, int max_wg, double* d_out,
                             hipStream_t s);
hipError_t launch_size_combine(const Mesh& m, double eps1, const double* sc, const double* gw,
                               double* gbeam, double* gquad, hipStream_t s);
hipError_t launch_hat_filter(int n, const int32_t* nodes, const Mesh& m, const double* g,
                             double r, double* out, unsigned* err, hipStream_t s);
hipError_t launch_gather(const Mesh& m, const Pattern& pat, const double* gbeam,
                         const double* gquad, double* dg_dxyz, double* dg_dt, double* dg_dscale,
                         hipStream_t s);

// assemble.hip
hipError_t launch_assemble(const Mesh& m, const Pattern& pat, const double* coo, double* K,
                           hipStream_t s);
hipError_t launch_loads(const Mesh& m, const Pattern& pat, const double* qarea, double* f,
                        hipStream_t s);
hipError_t launch_block_jacobi(const Mesh& m, const Pattern& pat, const double* K, double* Dinv,
                               float* Dinv32, unsigned* d_err, hipStream_t s);
// Lifting of prescribed displacements: f = 0 on constrained DOFs, fm - K_fc b on free ones;
// after the solve u = b on constrained DOFs.
hipError_t launch_lift(const Mesh& m, const Pattern& pat, const double* coo, const double* fm,
                       double* f, hipStream_t s);
hipError_t launch_apply_prescribed(const Mesh& m, double* u, hipStream_t s);
hipError_t launch_mask_vector(const Mesh& m, const double* in, double* out, hipStream_t s);
hipError_t launch_scalar_values(const Mesh& m, const Pattern& pat, const double* K,
                                double* vals, hipStream_t s);

// pcg.hip
struct PcgWork {
  int64_t n_dof = 0;
  int n_wg = 0;            // workgroups of the standard PCG kernels (grid-stride over the rows)
  int n_wg_f = 0;          // workgroups of the single-reduction kernels
  double* r = nullptr;
  double* z = nullptr;
  double* p[2] = {nullptr, nullptr};
  double* Ap = nullptr;
  double* xc = nullptr;          // FP64 correction solve: solution and residual
  double* rc = nullptr;
  double* fw[2] = {nullptr, nullptr};    // single-reduction variant: w = B r (on first use)
  float* fw32[2] = {nullptr, nullptr};
  int32_t* jw = nullptr;                  // per-workgroup iteration counters
  void* fdesc64 = nullptr;
  void* fdesc32 = nullptr;
  double* partials = nullptr;   // per-workgroup partial sums (see pcg.hip)
  PcgState* st = nullptr;
  PcgState* h_st = nullptr;     // host mirror
  PcgState* h_ring = nullptr;   // pinned [2]: state read-backs of consecutive polled chunks
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  // mixed precision: FP32 inner PCG vectors (allocated on first use)
  float* r32 = nullptr;
  float* z32 = nullptr;
  float* p32[2] = {nullptr, nullptr};
  float* Ap32 = nullptr;
  float* x32 = nullptr;
  float* b32 = nullptr;
  void* desc64 = nullptr;        // device descriptors of single-problem launches
  void* desc32 = nullptr;
  // sampled SpMV timing (HIP event pairs, created on first use)
  hipEvent_t* prof_ev = nullptr;
  int prof_cap = 0;
  double prof_us = 0.0;          // summed duration of the sampled launches of the last solve
  int prof_n = 0;
};

hipError_t pcg_alloc(PcgWork& w, int64_t n_nodes, bool mixed, hipStream_t s);
hipError_t pcg_alloc_mixed(PcgWork& w, hipStream_t s);
void pcg_free(PcgWork& w, const Arena* owner, hipStream_t s);  // owner: the problem's arena
// Solve K x = b (b already masked); x overwritten.  Returns SSO status via *status.
// profile_every > 0 times every n-th SpMV launch with HIP events (w.prof_us, w.prof_n).
// B = K Dinv (launch_right_precondition) selects the single-reduction recurrences, B = nullptr
// the standard ones.
// The standard recurrences on one workgroup (k_pcg_wg), all iterations in one launch (up to
// 16,384), then the same FP64 correction as pcg_solve.
hipError_t pcg_solve_wg(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                        const double* b, double* x, double rtol, int max_it, PcgWork& w,
                        hipStream_t s, int* iters, int* status, int profile_every);
hipError_t pcg_solve(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                     const double* B, const double* b, double* x, double rtol, int max_it,
                     PcgWork& w, hipStream_t s, int* iters, int* status, int profile_every = 0);
// The recurrences that run for an sso_options.solver value (AUTO resolved by size; the
// one-workgroup solver only in FP64).
int pcg_pick_solver(int solver, int64_t n_nodes, int64_t n_blocks, bool mixed);
// B = K Dinv block by block (B32: the same rounded to FP32; either may be null), in the padded
// block-row layout when the pattern has one; B holds right_precondition_blocks() 6x6 blocks.
int64_t right_precondition_blocks(const Pattern& pat, int64_t n_nodes);
hipError_t launch_right_precondition(const Mesh& m, const Pattern& pat, const double* K,
                                     const double* Dinv, double* B, float* B32, hipStream_t s);
// FP32 inner PCG inside FP64 iterative refinement (residual recomputed with the FP64 K); the
// inner solves use the single-reduction recurrences when B32 is given, else K32.
struct MixedParams {
  double rtol, inner_rtol;
  int max_it, refine_steps, inner_max_it;
};
struct MixedState {
  int outer = 0, iters = 0, status = SSO_OK;
  int k = 0, restarts = 0;    // outer steps since the last (re)start; restarts so far
  double rn = 0.0, bn = 0.0;  // |r| of the running inner solve's right-hand side; |b|
  bool done = false;
  FusedDesc<float> fdesc{};   // descriptor of the running inner solve: B32 given
  PcgDesc<float> sdesc{};     //   or the standard recurrences on K32
};
hipError_t pcg_solve_mixed(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                           const float* Dinv32, const float* B32, const double* b, double* x,
                           const MixedParams& mp, PcgWork& w, hipStream_t s, int* iters,
                           int* status, int* outer, int profile_every);
// The same one step at a time: mixed_begin sets x = 0 and starts the first inner solve (or
// stops at once); after the inner solve's state says done, mixed_step refines x and starts the
// next one or stops (ms.done, ms.status).  Both synchronise the stream.
hipError_t mixed_begin(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                       const float* Dinv32, const float* B32, const double* b, double* x,
                       const MixedParams& mp, PcgWork& w, hipStream_t s, MixedState& ms);
hipError_t mixed_step(const Mesh& m, const Pattern& pat, const double* K, const float* K32,
                      const float* Dinv32, const float* B32, const double* b, double* x,
                      const MixedParams& mp, PcgWork& w, hipStream_t s, MixedState& ms);
hipError_t launch_convert_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s);
// FP64 refinement of a converged solve until the true residual meets rtol (see pcg.hip).
hipError_t pcg_correct(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                       const double* b, double* x, double rtol, int max_it, PcgWork& w,
                       hipStream_t s, int* iters, int* status);

// Multi-problem iteration: problems started with pcg_begin (standard recurrences) or
// fused_begin (single-reduction) advance together, one launch per kernel for all problems of a
// kind (FP64).  A table lays the problems' workgroups end to end.
template <class Desc>
struct LaunchTable {
  void* d_desc = nullptr;
  int cap_desc = 0;
  int32_t* d_wg = nullptr;
  int cap_wg = 0;
  std::vector<Desc> h_desc;
  std::vector<int32_t> h_wg;
  int total = 0;          // workgroups of one launch
  bool lean = false;      // fused tables: every problem fits the lean multi-problem kernel
  bool sym = false;       // standard FP64 tables: the products read K's upper triangle
};
struct BatchWork {
  LaunchTable<PcgDesc<double>> standard;
  std::map<int, LaunchTable<FusedDesc<double>>> fused;   // by padded width
  LaunchTable<PcgDesc<float>> standard32;   // FP32 inner solves of mixed-precision problems
  LaunchTable<PcgDesc<double>> standard_upd;   // the k_update launches of the two above
  LaunchTable<PcgDesc<float>> standard32_upd;
  std::map<int, LaunchTable<FusedDesc<float>>> fused32;
  LaunchTable<PcgDesc<double>> wg;   // one-workgroup problems, launched on s_wg
  hipStream_t s_wg = nullptr;
  hipEvent_t ev_in = nullptr, ev_wg = nullptr;
  PcgState** d_stp = nullptr;
  int cap_stp = 0;
  PcgState* d_states = nullptr;
  int cap_states = 0;
  std::vector<PcgState*> h_stp;
  std::vector<PcgState> h_states;
  int64_t launched = 0;
  // asynchronous form: the states of the launched problems land in pinned memory, and an event
  // marks when they are there
  PcgState* h_pin = nullptr;
  int cap_pin = 0;
  hipEvent_t ev = nullptr;
  int pending_nt = -1;    // problems of the launch not yet waited for (-1: none pending)
  // timing samples (sso_batch_profile): time_span > 0 brackets the first time_span iterations of
  // the next launch with ev_t0 / ev_t1 on the launch stream
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
  int time_span = 0;
};
hipError_t pcg_begin(const Mesh& m, const Pattern& pat, const double* K, const double* Dinv,
                     const double* b, double* x, double rtol, int max_it, PcgWork& w,
                     hipStream_t s, PcgDesc<double>* desc);
hipError_t fused_begin(const Mesh& m, const Pattern& pat, const double* B, const double* Dinv,
                       const double* b, double* x, double rtol, int max_it, PcgWork& w,
                       hipStream_t s, FusedDesc<double>* desc);
// Descriptors of the problems of one multi-problem launch, by kind.
struct BatchLists {
  std::vector<PcgDesc<double>> standard;
  std::vector<FusedDesc<double>> fused;
  std::vector<PcgDesc<float>> standard32;   // FP32 inner solves of mixed precision
  std::vector<FusedDesc<float>> fused32;
  std::vector<PcgDesc<double>> wg;          // one workgroup per problem (k_pcg_wg), n_wg = 1
};
// The same in two halves: pcg_batch_launch enqueues the iterations and the copy of the states to
// pinned host memory and returns; pcg_batch_wait waits for them and fills bw.h_states.
hipError_t pcg_batch_launch(const BatchLists& lists, int n_iter, BatchWork& bw, hipStream_t s);
hipError_t pcg_batch_wait(BatchWork& bw);
// Launch n_iter iterations for every listed problem, one launch per kernel and kind, then copy
// their state records into bw.h_states in list order (standard, fused, standard32, fused32;
// synchronises the stream).
hipError_t pcg_batch_iterate(const BatchLists& lists, int n_iter, BatchWork& bw, hipStream_t s);
void batch_free(BatchWork& bw, hipStream_t s);
// Deterministic dot product a^T b; result written to *d_out (device).
hipError_t launch_dot(const double* a, const double* b, int64_t n, PcgWork& w, double* d_out,
                      hipStream_t s);
// r = b - K x (row sums in double-double, rounded to FP64 once), and rr = ||r||^2,
// bb = ||b||^2 into d_out[0], d_out[1].
hipError_t launch_true_residual(const Mesh& m, const Pattern& pat, const double* K,
                                const double* x, const double* b, double* r, PcgWork& w,
                                double* d_out, hipStream_t s);
// Single standard FP64 solves of a K of at least 128 MiB read only its upper triangle.
bool pcg_sym_products(int64_t n_blocks, bool mixed);
double pcg_bytes_per_iteration(int64_t n_nodes, int64_t n_blocks, bool mixed, bool sym);
double spmv_bytes_per_launch(int64_t n_nodes, int64_t n_blocks, bool mixed, bool sym);
double fused_bytes_per_iteration(int64_t n_nodes, int64_t n_blocks, bool mixed);

}  // namespace sso
