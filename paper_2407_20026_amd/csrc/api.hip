// C ABI and host runtime of libhipsso: problem lifecycle, device buffers, launch sequencing on
// the problem's stream, error mapping and per-stage timing.
#include <new>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "sso_internal.h"

using namespace sso;

// The static scratch of sso_size_objective_noalloc: one copy per device, for the life of the
// process.  In host code `scratch` names a host-side stand-in, not device memory; its device
// address on each GPU comes from hipGetSymbolAddress (taken once per device, with that device
// current) and only that address is ever handed to kernels.
static __device__ __align__(256) double scratch[SSO_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static_assert(SSO_NOALLOC_MAX_QUADS * 15 + 2 * 1024 <=
                  (int64_t)(SSO_NOALLOC_SCRATCH_BYTES / sizeof(double)),
              "the no-allocation scratch holds the partials and 15 values per quad");

// A block pattern shared by the problems of one topology (sso_problem_create_like); the last
// problem to be destroyed frees it.
struct SharedPattern {
  Pattern pat;
  std::atomic<int> refs{1};
};

struct sso_problem {
  hipStream_t s = nullptr;
  Mesh m;
  Pattern pat;                  // the pattern's arrays (owned through `shared`)
  SharedPattern* shared = nullptr;
  Arena mem;                    // chunks holding the problem's own device buffers
  sso_options opt;
  int64_t n_coo = 0;
  double* coo = nullptr;
  double* qarea = nullptr;
  double* K = nullptr;
  double* Dinv = nullptr;
  double* B = nullptr;          // K times the block-Jacobi inverse (single-reduction PCG)
  float* B32 = nullptr;
  float* K32 = nullptr;         // mixed precision copies (allocated on first mixed solve)
  float* Dinv32 = nullptr;
  double* f = nullptr;          // right-hand side of the masked system (lifted when prescribed)
  double* fm = nullptr;         // applied load on the free DOFs, when displacements are prescribed
  double* u = nullptr;
  double* lam = nullptr;
  double* rhs = nullptr;
  double* gbeam = nullptr;
  double* gquad = nullptr;
  double* gw = nullptr;         // size objective: volume terms [14 n_quads], shares [n_quads],
  double* wv = nullptr;         //   partials (allocated on first use)
  double* xpart = nullptr;
  double* d_scal = nullptr;     // small device scalars (dot products, residual norms)
  double* h_scal = nullptr;     // host mirror of d_scal (pageable)
  unsigned* d_err = nullptr;
  unsigned* h_err = nullptr;    // host mirror of d_err (pageable)
  PcgWork w;
  int32_t* row_ptr = nullptr;   // scalar CSR view (built on demand)
  int32_t* col = nullptr;
  int32_t* perm = nullptr;
  int32_t* seg = nullptr;
  bool solved = false;
  bool in_batch = false;        // started with sso_solve_begin, not yet finished
  bool batch_pending = false;   // listed in a multi-problem launch not yet waited for
  hipEvent_t ev_move = nullptr; // orders a new stream after the old one (sso_problem_set_stream)
  int solver_used = SSO_SOLVER_STANDARD;   // recurrences of the last solve
  PcgDesc<double> desc{};       // its descriptor in multi-problem launches (standard / fused)
  FusedDesc<double> fdesc{};
  MixedState ms;                // mixed precision begun with sso_solve_begin
  hipEvent_t ev[6] = {};
  int device = 0;               // the device current at creation (holds the problem's memory)
  int64_t bytes = 0;            // device memory allocated for the problem (sso_problem_bytes)
};

struct sso_batch {
  hipStream_t s = nullptr;
  BatchWork bw;
  bool pending = false;                  // a launch not yet waited for
  std::vector<sso_problem*> listed;      // its problem list, in the caller's order
  std::vector<int> idx[5];               // positions in that list by launch kind
  // sso_batch_profile: timing samples of the FP64 standard iterations
  int prof_every = 0, prof_span = 0;
  int64_t prof_calls = 0;                // launches that could be sampled so far
  int armed = 0;                         // iterations timed in the pending launch (0: none)
  std::vector<int> jn0;                  // its FP64 standard problems' next iteration index
  double prof_us = 0.0, prof_bytes = 0.0, prof_bytes_read = 0.0;
  int64_t prof_iters = 0;
};

namespace {

sso_options default_options() {
  sso_options o;
  o.precision = SSO_PREC_FP64;
  o.rtol = 1e-8;
  o.max_it = 200000;
  o.refine_steps = 20;
  o.profile_every = 0;
  o.inner_rtol = 0.0;
  o.solver = SSO_SOLVER_AUTO;
  o.inner_max_it = 0;
  return o;
}

bool options_ok(const sso_options& o) {
  return (o.precision == SSO_PREC_FP64 || o.precision == SSO_PREC_MIXED ||
          o.precision == SSO_PREC_AUTO) && o.rtol >= 0.0 &&
         o.max_it > 0 && o.refine_steps >= 0 && o.profile_every >= 0 && o.inner_rtol >= 0.0 &&
         o.inner_rtol < 1.0 && o.solver >= SSO_SOLVER_AUTO && o.solver <= SSO_SOLVER_WG &&
         o.inner_max_it >= 0 && !(o.solver == SSO_SOLVER_WG && o.precision == SSO_PREC_MIXED);
}

// The precision a problem runs in: AUTO resolves by the size of its FP64 K.
bool mixed_for(const sso_options& o, int64_t n_blocks) {
  if (o.solver == SSO_SOLVER_WG) return false;   // the one-workgroup solver runs in FP64
  if (o.precision == SSO_PREC_AUTO) {
    const double k_bytes = 288.0 * (double)n_blocks;
    return k_bytes >= (o.rtol <= SSO_AUTO_TIGHT_RTOL ? SSO_AUTO_MIXED_TIGHT_K_BYTES
                                                    : SSO_AUTO_MIXED_K_BYTES);
  }
  return o.precision == SSO_PREC_MIXED;
}

__global__ void k_fill(int64_t n, double v, double* out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}


int map_hip(hipError_t e) {
  if (e == hipSuccess) return SSO_OK;
  if (e == hipErrorOutOfMemory) return SSO_ENOMEM;
  return SSO_EHIP;
}

#define TRY_HIP(x)                     \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return map_hip(e_); \
  } while (0)

float elapsed_us(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return 1000.f * ms;
}

void free_problem(sso_problem* p) {
  if (!p) return;
  hipStream_t s = p->s;
  Mesh& m = p->m;
  for (void* q : {(void*)m.xyz, (void*)m.fixed, (void*)m.f_nodal, (void*)m.beam_nodes,
                  (void*)m.beam_prop, (void*)m.quad_nodes, (void*)m.quad_prop,
                  (void*)m.quad_scale, (void*)p->coo, (void*)p->qarea, (void*)p->K,
                  (void*)p->Dinv, (void*)p->f, (void*)p->K32, (void*)p->Dinv32, (void*)p->B, (void*)p->B32, (void*)p->u,
                  (void*)p->lam, (void*)p->rhs, (void*)p->gbeam, (void*)p->gquad,
                  (void*)p->d_scal, (void*)p->d_err, (void*)p->row_ptr, (void*)p->col,
                  (void*)p->perm, (void*)p->seg, (void*)m.u_presc, (void*)p->fm,
                  (void*)p->gw, (void*)p->wv, (void*)p->xpart})
    dev_release(q, &p->mem, s);
  if (p->shared) {
    if (p->shared->refs.fetch_sub(1) == 1) {   // the last problem of this topology
      free_pattern(p->shared->pat, s);
      delete p->shared;
    }
  } else {
    free_pattern(p->pat, s);
  }
  pcg_free(p->w, &p->mem, s);
  arena_free(p->mem, s);
  delete[] p->h_scal;
  delete p->h_err;
  for (auto& e : p->ev)
    if (e) (void)hipEventDestroy(e);
  if (p->ev_move) (void)hipEventDestroy(p->ev_move);
  (void)hipStreamSynchronize(s);
  delete p;
}

// Debug mode (HIPSSO_DEBUG set, and not "0", when a problem is created): the block pattern, the
// sort permutation and the padded rows built on the GPU are copied to the host and checked
// invariant by invariant (check_pattern); a failure is reported on stderr and as SSO_EINVAL.
bool debug_mode() {
  const char* v = std::getenv("HIPSSO_DEBUG");
  return v && *v && !(v[0] == '0' && v[1] == '\0');
}

int debug_check_pattern(sso_problem* p) {
  const Mesh& m = p->m;
  const Pattern& pat = p->pat;
  hipStream_t s = p->s;
  const int n = m.n_nodes;
  const int64_t nb = pat.n_blocks, nc = pat.n_bcoo;
  std::vector<int32_t> brow(n + 1), bcol(nb), bseg(nb + 1), bperm(nc), bslot(nc), bdiag(n),
      bsrow(nb), bsym(2 * nb), est(n + 1), ell((int64_t)n * pat.ell_w), bn(2 * (int64_t)m.n_beams),
      qn(4 * (int64_t)m.n_quads);
  auto get = [&](std::vector<int32_t>& v, const int32_t* src) {
    return v.empty() ? hipSuccess
                     : hipMemcpyAsync(v.data(), src, sizeof(int32_t) * v.size(),
                                      hipMemcpyDeviceToHost, s);
  };
  TRY_HIP(get(brow, pat.brow_ptr));
  TRY_HIP(get(bcol, pat.bcol));
  TRY_HIP(get(bseg, pat.bseg));
  TRY_HIP(get(bperm, pat.bperm));
  TRY_HIP(get(bslot, pat.bslot));
  TRY_HIP(get(bdiag, pat.bdiag));
  TRY_HIP(get(bsrow, pat.bsrow));
  TRY_HIP(get(bsym, pat.bsym));
  TRY_HIP(get(est, pat.estart));
  TRY_HIP(get(ell, pat.bcol_ell));
  TRY_HIP(get(bn, m.beam_nodes));
  TRY_HIP(get(qn, m.quad_nodes));
  TRY_HIP(hipStreamSynchronize(s));
  HostPattern h;
  h.n_nodes = n;
  h.n_beams = m.n_beams;
  h.n_quads = m.n_quads;
  h.ell_w = pat.ell_w;
  h.n_blocks = nb;
  h.n_bcoo = nc;
  h.brow_ptr = brow.data();
  h.bcol = bcol.data();
  h.bseg = bseg.data();
  h.bperm = bperm.data();
  h.bslot = bslot.data();
  h.bdiag = bdiag.data();
  h.bsrow = bsrow.data();
  h.bsym = bsym.data();
  h.estart = est.data();
  h.bcol_ell = ell.data();
  h.beam_nodes = bn.data();
  h.quad_nodes = qn.data();
  char msg[256];
  if (check_pattern(h, msg, sizeof msg) != 0) {
    std::fprintf(stderr, "hipsso debug: %s\n", msg);
    return SSO_EINVAL;
  }
  return SSO_OK;
}

// 1 in *err where two connectivity arrays of n entries differ.
__global__ void k_same_topology(int64_t n, const int32_t* a, const int32_t* b, unsigned* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && a[i] != b[i]) atomicOr(err, ERR_TOPO);
}

int create_impl(const sso_mesh* mesh, const sso_options* opts, hipStream_t stream,
                sso_problem* p, const sso_problem* like) {
  p->s = stream;
  TRY_HIP(hipGetDevice(&p->device));
  p->opt = opts ? *opts : default_options();
  Mesh& m = p->m;
  m.n_nodes = mesh->n_nodes;
  m.n_beams = mesh->n_beams;
  m.n_quads = mesh->n_quads;
  m.unit_weight = mesh->unit_weight;
  m.surface_load = mesh->surface_load;
  const int64_t nn = m.n_nodes, nb = m.n_beams, nq = m.n_quads;
  hipStream_t s = p->s;
  TRY_HIP(dev_alloc(&m.xyz, 3 * nn, s));
  TRY_HIP(dev_alloc(&m.fixed, 6 * nn, s));
  TRY_HIP(dev_alloc(&m.f_nodal, 6 * nn, s));
  TRY_HIP(dev_alloc(&m.beam_nodes, 2 * nb, s));
  TRY_HIP(dev_alloc(&m.beam_prop, 6 * nb, s));
  TRY_HIP(dev_alloc(&m.quad_nodes, 4 * nq, s));
  TRY_HIP(dev_alloc(&m.quad_prop, 5 * nq, s));
  TRY_HIP(dev_alloc(&m.quad_scale, nq, s));
  if (mesh->u_prescribed) {
    TRY_HIP(dev_alloc(&m.u_presc, 6 * nn, s));
    TRY_HIP(hipMemcpyAsync(m.u_presc, mesh->u_prescribed, sizeof(double) * 6 * nn,
                           hipMemcpyDeviceToDevice, s));
    TRY_HIP(dev_alloc(&p->fm, 6 * nn, s));
  }
  TRY_HIP(hipMemcpyAsync(m.xyz, mesh->xyz, sizeof(double) * 3 * nn, hipMemcpyDeviceToDevice, s));
  TRY_HIP(hipMemcpyAsync(m.fixed, mesh->fixed, 6 * nn, hipMemcpyDeviceToDevice, s));
  TRY_HIP(hipMemcpyAsync(m.f_nodal, mesh->f_nodal, sizeof(double) * 6 * nn,
                         hipMemcpyDeviceToDevice, s));
  if (nb) {
    TRY_HIP(hipMemcpyAsync(m.beam_nodes, mesh->beam_nodes, sizeof(int32_t) * 2 * nb,
                           hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipMemcpyAsync(m.beam_prop, mesh->beam_prop, sizeof(double) * 6 * nb,
                           hipMemcpyDeviceToDevice, s));
  }
  if (nq) {
    TRY_HIP(hipMemcpyAsync(m.quad_nodes, mesh->quad_nodes, sizeof(int32_t) * 4 * nq,
                           hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipMemcpyAsync(m.quad_prop, mesh->quad_prop, sizeof(double) * 5 * nq,
                           hipMemcpyDeviceToDevice, s));
    if (mesh->quad_scale) {
      TRY_HIP(hipMemcpyAsync(m.quad_scale, mesh->quad_scale, sizeof(double) * nq,
                             hipMemcpyDeviceToDevice, s));
    } else {
      hipLaunchKernelGGL(k_fill, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, nq, 1.0,
                         m.quad_scale);
      TRY_HIP(hipGetLastError());
    }
  }
  TRY_HIP(dev_alloc(&p->d_err, 1, s));
  p->h_err = new unsigned(0);
  TRY_HIP(dev_alloc(&p->d_scal, 8, s));
  p->h_scal = new double[8]();
  TRY_HIP(hipMemsetAsync(p->d_err, 0, sizeof(unsigned), s));
  *p->h_err = 0;
  if (like) {
    // the pattern of `like`, once its connectivity is shown to be this mesh's (checked with the
    // other errors at the end of creation)
    p->pat = like->pat;
    p->shared = like->shared;
    p->shared->refs.fetch_add(1);
    const int64_t nbn = 2 * (int64_t)nb, nqn = 4 * (int64_t)nq;
    if (nbn)
      hipLaunchKernelGGL(k_same_topology, dim3((unsigned)((nbn + 255) / 256)), dim3(256), 0, s,
                         nbn, m.beam_nodes, like->m.beam_nodes, p->d_err);
    if (nqn)
      hipLaunchKernelGGL(k_same_topology, dim3((unsigned)((nqn + 255) / 256)), dim3(256), 0, s,
                         nqn, m.quad_nodes, like->m.quad_nodes, p->d_err);
    TRY_HIP(hipGetLastError());
  } else {
    {
      AllocScope ps(&p->bytes, &p->pat.mem);   // the pattern outlives this problem if shared
      TRY_HIP(build_pattern(m, p->pat, p->d_err, s, p->h_err));
    }
    if (*p->h_err) return SSO_EINVAL;
    p->shared = new (std::nothrow) SharedPattern();
    if (!p->shared) return SSO_ENOMEM;
    p->shared->pat = p->pat;
    if (debug_mode()) {
      const int st = debug_check_pattern(p);
      if (st != SSO_OK) return st;
    }
  }
  p->n_coo = 144 * nb + 576 * nq;
  TRY_HIP(dev_alloc(&p->coo, p->n_coo, s));
  TRY_HIP(dev_alloc(&p->qarea, nq, s));
  TRY_HIP(dev_alloc(&p->K, 36 * p->pat.n_blocks, s));
  TRY_HIP(dev_alloc(&p->Dinv, dinv_packed_len(nn), s));
  TRY_HIP(dev_alloc(&p->f, 6 * nn, s));
  TRY_HIP(dev_alloc(&p->u, 6 * nn, s));
  TRY_HIP(dev_alloc(&p->lam, 6 * nn, s));
  TRY_HIP(dev_alloc(&p->rhs, 6 * nn, s));
  TRY_HIP(dev_alloc(&p->gbeam, 6 * nb, s));
  TRY_HIP(dev_alloc(&p->gquad, 14 * nq, s));
  TRY_HIP(pcg_alloc(p->w, nn, mixed_for(p->opt, p->pat.n_blocks), s));
  for (auto& e : p->ev) TRY_HIP(hipEventCreate(&e));
  if (like) TRY_HIP(hipMemcpyAsync(p->h_err, p->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (like && *p->h_err) return SSO_EINVAL;
  return SSO_OK;
}

int read_errors(sso_problem* p) {
  TRY_HIP(hipMemcpyAsync(p->h_err, p->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, p->s));
  TRY_HIP(hipStreamSynchronize(p->s));
  return *p->h_err ? SSO_EINVAL : SSO_OK;
}

}  // namespace

extern "C" {

int sso_problem_create(const sso_mesh* mesh, const sso_options* opts, hipStream_t stream,
                       sso_problem** out) {
  if (!mesh || !out) return SSO_EINVAL;
  *out = nullptr;
  if (mesh->n_nodes <= 0 || mesh->n_beams < 0 || mesh->n_quads < 0) return SSO_EINVAL;
  if (!mesh->xyz || !mesh->fixed || !mesh->f_nodal) return SSO_EINVAL;
  if (mesh->n_beams > 0 && (!mesh->beam_nodes || !mesh->beam_prop)) return SSO_EINVAL;
  if (mesh->n_quads > 0 && (!mesh->quad_nodes || !mesh->quad_prop)) return SSO_EINVAL;
  if (16 * (int64_t)mesh->n_quads + 4 * (int64_t)mesh->n_beams >= (int64_t)1 << 31)
    return SSO_EINVAL;
  if (opts && !options_ok(*opts)) return SSO_EINVAL;
  sso_problem* p = new (std::nothrow) sso_problem();
  if (!p) return SSO_ENOMEM;
  AllocScope ac(&p->bytes, &p->mem);
  int st = create_impl(mesh, opts, stream, p, nullptr);
  if (st != SSO_OK) {
    free_problem(p);
    return st;
  }
  *out = p;
  return SSO_OK;
}

int sso_problem_create_like(const sso_problem* like, const sso_mesh* mesh,
                            const sso_options* opts, hipStream_t stream, sso_problem** out) {
  if (!like || !mesh || !out) return SSO_EINVAL;
  *out = nullptr;
  if (mesh->n_nodes != like->m.n_nodes || mesh->n_beams != like->m.n_beams ||
      mesh->n_quads != like->m.n_quads)
    return SSO_EINVAL;
  if (!mesh->xyz || !mesh->fixed || !mesh->f_nodal) return SSO_EINVAL;
  if (mesh->n_beams > 0 && (!mesh->beam_nodes || !mesh->beam_prop)) return SSO_EINVAL;
  if (mesh->n_quads > 0 && (!mesh->quad_nodes || !mesh->quad_prop)) return SSO_EINVAL;
  if (opts && !options_ok(*opts)) return SSO_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != like->device) return SSO_EINVAL;
  sso_problem* p = new (std::nothrow) sso_problem();
  if (!p) return SSO_ENOMEM;
  AllocScope ac(&p->bytes, &p->mem);
  int st = create_impl(mesh, opts, stream, p, like);
  if (st != SSO_OK) {
    free_problem(p);
    return st;
  }
  *out = p;
  return SSO_OK;
}

int sso_problem_update(sso_problem* p, const double* xyz, const double* quad_t,
                       const double* quad_scale) {
  if (!p) return SSO_EINVAL;
  Mesh& m = p->m;
  if (xyz)
    TRY_HIP(hipMemcpyAsync(m.xyz, xyz, sizeof(double) * 3 * (size_t)m.n_nodes,
                           hipMemcpyDeviceToDevice, p->s));
  if (quad_t && m.n_quads)
    TRY_HIP(hipMemcpy2DAsync(m.quad_prop, 5 * sizeof(double), quad_t, sizeof(double),
                             sizeof(double), (size_t)m.n_quads, hipMemcpyDeviceToDevice, p->s));
  if (quad_scale && m.n_quads)
    TRY_HIP(hipMemcpyAsync(m.quad_scale, quad_scale, sizeof(double) * (size_t)m.n_quads,
                           hipMemcpyDeviceToDevice, p->s));
  p->solved = false;
  return SSO_OK;
}

int sso_set_options(sso_problem* p, const sso_options* opts) {
  if (!p || !opts || !options_ok(*opts) || p->in_batch) return SSO_EINVAL;
  // K32 / B / B32 are built by sso_solve for the precision and recurrences it runs with
  if (opts->precision != p->opt.precision || opts->solver != p->opt.solver) p->solved = false;
  p->opt = *opts;
  return SSO_OK;
}

}  // extern "C"

namespace {

bool mixed(const sso_problem* p) { return mixed_for(p->opt, p->pat.n_blocks); }
bool fused(const sso_problem* p) { return p->solver_used == SSO_SOLVER_FUSED; }
bool one_wg(const sso_problem* p) { return p->solver_used == SSO_SOLVER_WG; }
// iteration of a begun problem has stopped (mixed precision: the refinement loop has)
bool stopped(const sso_problem* p) { return mixed(p) ? p->ms.done : p->w.h_st->done != 0; }

MixedParams mixed_params(const sso_problem* p) {
  MixedParams mp;
  mp.rtol = p->opt.rtol;
  mp.inner_rtol = p->opt.inner_rtol > 0.0 ? p->opt.inner_rtol : 1e-5;
  mp.max_it = p->opt.max_it;
  mp.refine_steps = p->opt.refine_steps;
  mp.inner_max_it = p->opt.inner_max_it;
  if (p->opt.precision == SSO_PREC_AUTO) {   // AUTO's mixed precision: capped inner solves
    constexpr int AUTO_INNER_CAP = 30;
    if (mp.inner_max_it == 0) mp.inner_max_it = AUTO_INNER_CAP;
    const int outer = p->opt.max_it / mp.inner_max_it + 1;
    if (mp.refine_steps < outer) mp.refine_steps = outer;
  }
  return mp;
}

// Solve K x = b (b masked) in the problem's precision mode.
int run_solver(sso_problem* p, const double* b, double* x, int* iters, int* outer) {
  int status = SSO_OK;
  *outer = 0;
  if (one_wg(p)) {
    TRY_HIP(pcg_solve_wg(p->m, p->pat, p->K, p->Dinv, b, x, p->opt.rtol, p->opt.max_it, p->w,
                         p->s, iters, &status, p->opt.profile_every));
  } else if (!mixed(p)) {
    TRY_HIP(pcg_solve(p->m, p->pat, p->K, p->Dinv, fused(p) ? p->B : nullptr, b, x, p->opt.rtol,
                      p->opt.max_it, p->w, p->s, iters, &status, p->opt.profile_every));
  } else {
    TRY_HIP(pcg_solve_mixed(p->m, p->pat, p->K, p->K32, p->Dinv32, fused(p) ? p->B32 : nullptr,
                            b, x, mixed_params(p), p->w, p->s, iters, &status, outer,
                            p->opt.profile_every));
  }
  return status;
}

// Elements, loads, assembly, masking, block-Jacobi and the operators the chosen PCG needs
// (B = K M for the single-reduction recurrences; FP32 copies for mixed precision).  Events 0-2
// bracket the stages.
int prepare(sso_problem* p, bool batch) {
  hipStream_t s = p->s;
  p->solver_used = pcg_pick_solver(p->opt.solver, p->m.n_nodes, p->pat.n_blocks,
                                   mixed_for(p->opt, p->pat.n_blocks));
  // multi-problem launches: many problems in flight make the iteration bandwidth-bound, where
  // the standard pair streams faster than the fused kernel (16 60 x 60 shells: 123 vs 93
  // solves/s; 256 80 x 80 shells: 13.2 vs 19.2 s).  A problem resident in one workgroup's LDS
  // keeps that solver in its kernel beside the launches (served stream: the small requests'
  // median latency 14.5 -> 5.1 ms at the same capacity).
  if (batch && p->opt.solver == SSO_SOLVER_AUTO && p->solver_used != SSO_SOLVER_WG)
    p->solver_used = SSO_SOLVER_STANDARD;
  const bool mx = mixed(p), fu = fused(p);
  const int64_t nk = 36 * p->pat.n_blocks;
  const int64_t nb = 36 * right_precondition_blocks(p->pat, p->m.n_nodes);
  if (mx && !p->Dinv32) TRY_HIP(dev_alloc(&p->Dinv32, dinv_packed_len(p->m.n_nodes), s));
  if (mx && !fu && !p->K32) TRY_HIP(dev_alloc(&p->K32, nk, s));
  if (fu && !mx && !p->B) TRY_HIP(dev_alloc(&p->B, nb, s));
  if (fu && mx && !p->B32) TRY_HIP(dev_alloc(&p->B32, nb, s));
  TRY_HIP(hipMemsetAsync(p->d_err, 0, sizeof(unsigned), s));
  TRY_HIP(hipEventRecord(p->ev[0], s));
  TRY_HIP(launch_element_stiffness(p->m, p->coo, p->qarea, p->d_err, s));
  if (p->fm) {
    TRY_HIP(launch_loads(p->m, p->pat, p->qarea, p->fm, s));
    TRY_HIP(launch_lift(p->m, p->pat, p->coo, p->fm, p->f, s));
  } else {
    TRY_HIP(launch_loads(p->m, p->pat, p->qarea, p->f, s));
  }
  TRY_HIP(hipEventRecord(p->ev[1], s));
  TRY_HIP(launch_assemble(p->m, p->pat, p->coo, p->K, s));
  TRY_HIP(launch_block_jacobi(p->m, p->pat, p->K, p->Dinv, mx ? p->Dinv32 : nullptr, p->d_err,
                              s));
  if (mx && !fu) TRY_HIP(launch_convert_f32(p->K, p->K32, nk, s));
  if (fu)
    TRY_HIP(launch_right_precondition(p->m, p->pat, p->K, p->Dinv, mx ? nullptr : p->B,
                                      mx ? p->B32 : nullptr, s));
  TRY_HIP(hipEventRecord(p->ev[2], s));
  return read_errors(p);
}

bool fused_used(const sso_problem* p) { return p->solver_used == SSO_SOLVER_FUSED; }

// single: a solve of its own (sso_solve, the adjoint), whose standard FP64 products read only
// K's upper triangle above the size pcg_sym_products names; multi-problem launches read all of K
bool sym_used(const sso_problem* p, bool single) {
  return single && p->solver_used == SSO_SOLVER_STANDARD && pcg_sym_products(p->pat.n_blocks, mixed(p));
}

double solve_bytes(const sso_problem* p, int iters, int outer, bool single) {
  const int64_t nn = p->m.n_nodes, nb = p->pat.n_blocks;
  if (fused_used(p) && !mixed(p)) return iters * fused_bytes_per_iteration(nn, nb, false);
  if (!mixed(p)) return iters * pcg_bytes_per_iteration(nn, nb, false, sym_used(p, single));
  // inner FP32 iterations + one FP64 residual SpMV (K, x, b read; r written) per outer step
  double resid = 292.0 * nb + 4.0 * (nn + 1) + 3.0 * 8.0 * 6.0 * nn;
  return iters * pcg_bytes_per_iteration(nn, nb, true, false) + (outer + 1) * resid;
}

// ---- penalised volume objective (Sec. 3.3): shared by the allocating and static-scratch forms

constexpr int SIZE_XWG = 1024;   // workgroups (partials) of the size-objective reduction

bool size_args_ok(const sso_problem* p, double eps1, double u_max, double t_min,
                  const double* out_host, const double* dg_dxyz) {
  return p && p->solved && out_host && dg_dxyz && eps1 >= 0.0 && std::isfinite(eps1) &&
         u_max > 0.0 && std::isfinite(u_max) && t_min > 0.0 && std::isfinite(t_min);
}

// g = (1 + eps1 c) W and its gradient with the scratch arrays xpart [2 SIZE_XWG], gw
// [14 n_quads] and wv [n_quads] given.
int size_objective_impl(sso_problem* p, double eps1, double u_max, double t_min,
                        double* out_host, double* dg_dxyz, double* dg_dt, sso_stats* stats,
                        double* xpart, double* gw, double* wv) {
  hipStream_t s = p->s;
  const Mesh& m = p->m;
  TRY_HIP(hipEventRecord(p->ev[4], s));
  // volume terms, then dc/du (masked) with the sums c and W in d_scal[2..3]
  TRY_HIP(launch_volume_terms(m, t_min, gw, wv, s));
  TRY_HIP(launch_size_terms(m, p->u, u_max, wv, p->rhs, xpart, SIZE_XWG, p->d_scal + 2, s));
  int iters = 0, outer = 0;
  const int status = run_solver(p, p->rhs, p->lam, &iters, &outer);
  if (status != SSO_OK && status != SSO_ENOTCONV) return status;
  TRY_HIP(launch_adjoint_terms(m, p->pat, p->u, p->lam, 1.0, 0.0, p->gbeam, p->gquad, s));
  TRY_HIP(launch_size_combine(m, eps1, p->d_scal + 2, gw, p->gbeam, p->gquad, s));
  TRY_HIP(launch_gather(m, p->pat, p->gbeam, p->gquad, dg_dxyz, dg_dt, nullptr, s));
  TRY_HIP(hipEventRecord(p->ev[5], s));
  TRY_HIP(hipMemcpyAsync(p->h_scal + 2, p->d_scal + 2, 2 * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  const double c = p->h_scal[2], W = p->h_scal[3];
  out_host[0] = (1.0 + eps1 * c) * W;
  out_host[1] = c;
  out_host[2] = W;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = iters;
    stats->t_adj_us = elapsed_us(p->ev[4], p->ev[5]);
  }
  return status;
}

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_ptr[MAX_DEVICES] = {};

int scratch_address(int device, double** out) {
  if (device < 0 || device >= MAX_DEVICES) return SSO_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[device]) {
    int cur = 0;
    TRY_HIP(hipGetDevice(&cur));
    if (cur != device) TRY_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return map_hip(e);
    if (!ptr) return SSO_EHIP;
    scratch_ptr[device] = static_cast<double*>(ptr);
  }
  *out = scratch_ptr[device];
  return SSO_OK;
}


std::mutex pool_mutex;
hipMemPool_t pools[MAX_DEVICES] = {};

// The device's pool, created on first use with an unlimited release threshold.
hipError_t device_pool(int device, hipMemPool_t* out) {
  std::lock_guard<std::mutex> lock(pool_mutex);
  if (!pools[device]) {
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    hipError_t e = hipMemPoolCreate(&pool, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = UINT64_MAX;
    e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(pool);
      return e;
    }
    pools[device] = pool;
  }
  *out = pools[device];
  return hipSuccess;
}

}  // namespace

namespace sso {

// Every device buffer of the library comes from a pool of its own per device that keeps freed
// memory for the next allocation.  The default pool's release threshold of zero hands freed
// memory back to the driver at each synchronisation and the next allocation maps it afresh,
// which cost about 0.85 ms per destroyed problem and 1 ms per created one on the served sizes.
hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  int device = 0;
  hipError_t e = hipStreamGetDevice(s, &device);
  if (e != hipSuccess) return e;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  hipMemPool_t pool = nullptr;
  e = device_pool(device, &pool);
  if (e != hipSuccess) return e;
  return hipMallocFromPoolAsync(p, bytes, pool, s);
}

hipError_t arena_alloc(Arena& a, size_t bytes, hipStream_t s, void** out, int64_t* held) {
  bytes = (bytes + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
  *held = 0;
  if (bytes > ARENA_CHUNK / 4) {   // a chunk of its own
    void* q = nullptr;
    const hipError_t e = pool_alloc(&q, bytes, s);
    if (e != hipSuccess) return e;
    a.chunks.emplace_back(static_cast<char*>(q), bytes);
    *held = (int64_t)bytes;
    *out = q;
    return hipSuccess;
  }
  if (bytes > a.left) {
    void* q = nullptr;
    const hipError_t e = pool_alloc(&q, ARENA_CHUNK, s);
    if (e != hipSuccess) return e;
    a.chunks.emplace_back(static_cast<char*>(q), ARENA_CHUNK);
    a.cur = static_cast<char*>(q);
    a.left = ARENA_CHUNK;
    *held = (int64_t)ARENA_CHUNK;
  }
  *out = a.cur;
  a.cur += bytes;
  a.left -= bytes;
  return hipSuccess;
}

bool arena_owns(const Arena& a, const void* p) {
  const char* c = static_cast<const char*>(p);
  for (const auto& k : a.chunks)
    if (c >= k.first && c < k.first + k.second) return true;
  return false;
}

void arena_free(Arena& a, hipStream_t s) {
  for (const auto& k : a.chunks) (void)hipFreeAsync(k.first, s);
  a = Arena();
}

}  // namespace sso

extern "C" {

int sso_solve(sso_problem* p, double* u_out, sso_stats* stats) {
  if (!p) return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  hipStream_t s = p->s;
  p->solved = false;
  p->in_batch = false;
  int st = prepare(p, false);
  if (st != SSO_OK) return st;
  int iters = 0, outer = 0;
  int status = run_solver(p, p->f, p->u, &iters, &outer);
  if (status == SSO_EHIP || status == SSO_ENOMEM) return status;
  TRY_HIP(hipEventRecord(p->ev[3], s));
  TRY_HIP(launch_true_residual(p->m, p->pat, p->K, p->u, p->f, nullptr, p->w, p->d_scal, s));
  TRY_HIP(hipMemcpyAsync(p->h_scal, p->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (p->m.u_presc) TRY_HIP(launch_apply_prescribed(p->m, p->u, s));
  if (u_out)
    TRY_HIP(hipMemcpyAsync(u_out, p->u, sizeof(double) * 6 * (size_t)p->m.n_nodes,
                           hipMemcpyDeviceToDevice, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = iters;
    stats->refine_steps = outer;
    stats->rel_residual = p->h_scal[1] > 0 ? sqrt(p->h_scal[0] / p->h_scal[1]) : 0.0;
    stats->t_elem_us = elapsed_us(p->ev[0], p->ev[1]);
    stats->t_asm_us = elapsed_us(p->ev[1], p->ev[2]);
    stats->t_solve_us = elapsed_us(p->ev[2], p->ev[3]);
    stats->bytes_moved = solve_bytes(p, iters, outer, true);
    stats->spmv_samples = p->w.prof_n;
    stats->spmv_us = p->w.prof_n ? p->w.prof_us / p->w.prof_n : 0.0;
    stats->spmv_bytes =
        fused_used(p) ? fused_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, mixed(p))
                      : pcg_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, mixed(p),
                                                sym_used(p, true));
    stats->solver = p->solver_used;
    stats->sym_products = sym_used(p, true) ? 1 : 0;
  }
  // after SSO_ENOTCONV u holds the last iterate; objective and adjoint stay available
  p->solved = (status == SSO_OK || status == SSO_ENOTCONV);
  return status;
}

int sso_solve_begin(sso_problem* p) {
  if (!p) return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  // multi-problem launches run FP64 iterations of either kind and FP32 single-reduction ones
  hipStream_t s = p->s;
  p->solved = false;
  p->in_batch = false;
  int st = prepare(p, true);
  if (st != SSO_OK) return st;
  if (mixed(p))
    TRY_HIP(mixed_begin(p->m, p->pat, p->K, p->K32, p->Dinv32, p->B32, p->f, p->u,
                        mixed_params(p), p->w, s, p->ms));
  else if (fused(p))
    TRY_HIP(fused_begin(p->m, p->pat, p->B, p->Dinv, p->f, p->u, p->opt.rtol, p->opt.max_it,
                        p->w, s, &p->fdesc));
  else
    TRY_HIP(pcg_begin(p->m, p->pat, p->K, p->Dinv, p->f, p->u, p->opt.rtol, p->opt.max_it,
                      p->w, s, &p->desc));
  p->in_batch = true;
  return SSO_OK;
}

int sso_solve_end(sso_problem* p, double* u_out, sso_stats* stats) {
  if (!p || !p->in_batch || p->batch_pending) return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  hipStream_t s = p->s;
  TRY_HIP(hipMemcpyAsync(p->w.h_st, p->w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  TRY_HIP(launch_true_residual(p->m, p->pat, p->K, p->u, p->f, nullptr, p->w, p->d_scal, s));
  TRY_HIP(hipMemcpyAsync(p->h_scal, p->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  int status = p->w.h_st->done ? p->w.h_st->status : SSO_ENOTCONV;
  int iters = p->w.h_st->it, outer = 0;
  if (mixed(p)) {   // the refinement loop already ended on the FP64 true residual
    status = p->ms.done ? p->ms.status : SSO_ENOTCONV;
    iters = p->ms.iters;
    outer = p->ms.outer;
  } else if (status == SSO_OK) {
    TRY_HIP(pcg_correct(p->m, p->pat, p->K, p->Dinv, p->f, p->u, p->opt.rtol, p->opt.max_it, p->w,
                        s, &iters, &status));
    TRY_HIP(launch_true_residual(p->m, p->pat, p->K, p->u, p->f, nullptr, p->w, p->d_scal, s));
    TRY_HIP(hipMemcpyAsync(p->h_scal, p->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  if (p->m.u_presc) TRY_HIP(launch_apply_prescribed(p->m, p->u, s));
  if (u_out)
    TRY_HIP(hipMemcpyAsync(u_out, p->u, sizeof(double) * 6 * (size_t)p->m.n_nodes,
                           hipMemcpyDeviceToDevice, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = iters;
    stats->rel_residual = p->h_scal[1] > 0 ? sqrt(p->h_scal[0] / p->h_scal[1]) : 0.0;
    stats->refine_steps = outer;
    stats->bytes_moved = solve_bytes(p, iters, outer, false);
    stats->spmv_bytes =
        fused(p) ? fused_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, mixed(p))
                 : pcg_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, mixed(p), false);
    stats->solver = p->solver_used;
  }
  p->in_batch = false;
  p->solved = (status == SSO_OK || status == SSO_ENOTCONV);
  return status;
}

int sso_batch_create(hipStream_t stream, sso_batch** out) {
  if (!out) return SSO_EINVAL;
  sso_batch* b = new (std::nothrow) sso_batch();
  if (!b) return SSO_ENOMEM;
  b->s = stream;
  *out = b;
  return SSO_OK;
}

int sso_batch_launch(sso_batch* b, sso_problem* const* ps, int n, int n_iter) {
  if (!b || (n > 0 && !ps) || n < 0 || n_iter < 0 || b->pending) return SSO_EINVAL;
  for (int i = 0; i < n; ++i) {
    sso_problem* p = ps[i];
    if (!p || !p->in_batch || p->s != b->s || p->batch_pending) return SSO_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ps[k] == p) return SSO_EINVAL;   // a problem listed twice would advance twice
  }
  BatchLists lists;
  for (auto& v : b->idx) v.clear();
  for (int i = 0; i < n; ++i) {
    sso_problem* p = ps[i];
    if (stopped(p)) continue;          // finished at an earlier poll
    if (mixed(p) && fused(p)) {
      lists.fused32.push_back(p->ms.fdesc);
      b->idx[3].push_back(i);
    } else if (mixed(p)) {
      lists.standard32.push_back(p->ms.sdesc);
      b->idx[2].push_back(i);
    } else if (fused(p)) {
      lists.fused.push_back(p->fdesc);
      b->idx[1].push_back(i);
    } else if (one_wg(p)) {
      PcgDesc<double> d = p->desc;
      d.n_wg = 1;
      lists.wg.push_back(d);
      b->idx[4].push_back(i);
    } else {
      lists.standard.push_back(p->desc);
      b->idx[0].push_back(i);
    }
  }
  // a timing sample: every prof_every-th launch that holds FP64 standard problems and no other
  // kind on the batch stream (one-workgroup problems run on their own stream beside them)
  b->armed = 0;
  if (b->prof_every > 0 && n_iter > 0 && !lists.standard.empty() && lists.fused.empty() &&
      lists.standard32.empty() && lists.fused32.empty() &&
      b->prof_calls++ % b->prof_every == 0) {
    b->armed = b->prof_span < n_iter ? b->prof_span : n_iter;
    b->jn0.clear();
    for (int i : b->idx[0]) b->jn0.push_back(ps[i]->w.h_st->jn);
  }
  b->bw.time_span = b->armed;
  TRY_HIP(pcg_batch_launch(lists, n_iter, b->bw, b->s));
  b->listed.assign(ps, ps + n);
  for (int i = 0; i < n; ++i) ps[i]->batch_pending = true;
  b->pending = true;
  return SSO_OK;
}

int sso_batch_wait(sso_batch* b, sso_problem* const* ps, int n, int32_t* done) {
  if (!b || !b->pending || n != (int)b->listed.size() || (n > 0 && !ps)) return SSO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (ps[i] != b->listed[i]) return SSO_EINVAL;
  b->pending = false;
  for (int i = 0; i < n; ++i) ps[i]->batch_pending = false;
  TRY_HIP(pcg_batch_wait(b->bw));
  size_t k0 = 0;
  for (const auto& v : b->idx)
    for (int i : v) *ps[i]->w.h_st = b->bw.h_states[k0++];
  if (b->armed > 0) {
    // each problem's iterations inside the timed span: how far its next iteration index moved
    // (an iteration that finds the problem stopped does no work and does not move it), at most
    // the span; bytes per iteration with all of K counted, and as the launch's product read K
    const int span = b->armed;
    b->armed = 0;
    float ms = 0.0f;
    TRY_HIP(hipEventElapsedTime(&ms, b->bw.ev_t0, b->bw.ev_t1));
    b->prof_us += 1000.0 * (double)ms;
    b->prof_iters += span;
    const bool sym = b->bw.standard.sym;
    for (size_t k = 0; k < b->idx[0].size(); ++k) {
      const sso_problem* p = ps[b->idx[0][k]];
      int d = p->w.h_st->jn - b->jn0[k];
      d = d < 0 ? 0 : (d > span ? span : d);
      b->prof_bytes += d * pcg_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, false, false);
      b->prof_bytes_read += d * pcg_bytes_per_iteration(p->m.n_nodes, p->pat.n_blocks, false, sym);
    }
  }
  // mixed precision: a stopped inner solve is refined in FP64 and the next one started
  for (const std::vector<int>* v : {&b->idx[2], &b->idx[3]})
    for (int i : *v) {
      sso_problem* p = ps[i];
      TRY_HIP(mixed_step(p->m, p->pat, p->K, p->K32, p->Dinv32, p->B32, p->f, p->u,
                         mixed_params(p), p->w, p->s, p->ms));
    }
  if (done)
    for (int i = 0; i < n; ++i) done[i] = stopped(ps[i]) ? 1 : 0;
  return SSO_OK;
}

int sso_batch_iterate(sso_batch* b, sso_problem* const* ps, int n, int n_iter, int32_t* done) {
  const int st = sso_batch_launch(b, ps, n, n_iter);
  if (st != SSO_OK) return st;
  return sso_batch_wait(b, ps, n, done);
}

int sso_problem_set_stream(sso_problem* p, hipStream_t stream) {
  if (!p || p->batch_pending) return SSO_EINVAL;
  if (stream == p->s) return SSO_OK;
  if (!p->ev_move) TRY_HIP(hipEventCreateWithFlags(&p->ev_move, hipEventDisableTiming));
  TRY_HIP(hipEventRecord(p->ev_move, p->s));
  TRY_HIP(hipStreamWaitEvent(stream, p->ev_move, 0));
  p->s = stream;
  return SSO_OK;
}

int sso_batch_profile(sso_batch* b, int every, int span) {
  if (!b || every < 0 || span < 0 || (every > 0 && span == 0) || b->pending) return SSO_EINVAL;
  if (every > 0 && !b->bw.ev_t0) {
    int dev = 0, cur = 0;
    TRY_HIP(hipStreamGetDevice(b->s, &dev));
    TRY_HIP(hipGetDevice(&cur));
    if (cur != dev) TRY_HIP(hipSetDevice(dev));
    hipError_t e = hipEventCreate(&b->bw.ev_t0);
    if (e == hipSuccess) e = hipEventCreate(&b->bw.ev_t1);
    if (cur != dev) (void)hipSetDevice(cur);
    TRY_HIP(e);
  }
  b->prof_every = every;
  b->prof_span = span;
  b->prof_calls = 0;
  b->prof_us = b->prof_bytes = b->prof_bytes_read = 0.0;
  b->prof_iters = 0;
  return SSO_OK;
}

int sso_batch_timing(const sso_batch* b, double* us, int64_t* iters, double* bytes,
                     double* bytes_read) {
  if (!b) return SSO_EINVAL;
  if (us) *us = b->prof_us;
  if (iters) *iters = b->prof_iters;
  if (bytes) *bytes = b->prof_bytes;
  if (bytes_read) *bytes_read = b->prof_bytes_read;
  return SSO_OK;
}

void sso_batch_destroy(sso_batch* b) {
  if (!b) return;
  for (sso_problem* p : b->listed)   // a launch never waited for: its problems are free again
    if (b->pending && p) p->batch_pending = false;
  batch_free(b->bw, b->s);
  (void)hipStreamSynchronize(b->s);
  delete b;
}

int sso_objective(sso_problem* p, int kind, const double* a, double* g_host) {
  if (!p || !g_host || !p->solved) return SSO_EINVAL;
  const double* lhs;
  double scale = 1.0;
  const double* load = p->fm ? p->fm : p->f;
  if (kind == SSO_OBJ_COMPLIANCE) {
    lhs = load;
  } else if (kind == SSO_OBJ_STRAIN_ENERGY) {
    lhs = load;
    scale = 0.5;
  } else if (kind == SSO_OBJ_LINEAR && a) {
    lhs = a;
  } else {
    return SSO_EINVAL;
  }
  const int64_t n = 6 * (int64_t)p->m.n_nodes;
  TRY_HIP(launch_dot(lhs, p->u, n, p->w, p->d_scal, p->s));
  TRY_HIP(hipMemcpyAsync(p->h_scal, p->d_scal, sizeof(double), hipMemcpyDeviceToHost, p->s));
  TRY_HIP(hipStreamSynchronize(p->s));
  *g_host = scale * p->h_scal[0];
  return SSO_OK;
}

int sso_adjoint(sso_problem* p, int kind, const double* dg_du, double* dg_dxyz, double* dg_dt,
                double* dg_dscale, sso_stats* stats) {
  if (!p || !p->solved || !dg_dxyz) return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  hipStream_t s = p->s;
  double c_lam = 1.0, c_u = 1.0;
  const double* lam = p->u;
  int iters = 0, status = SSO_OK;
  TRY_HIP(hipEventRecord(p->ev[4], s));
  if (kind == SSO_OBJ_COMPLIANCE || kind == SSO_OBJ_STRAIN_ENERGY) {
    if (kind == SSO_OBJ_STRAIN_ENERGY) c_lam = c_u = 0.5;
    if (p->fm) {
      // prescribed displacements: u solves the lifted system, so K lambda = f needs a solve
      int outer = 0;
      status = run_solver(p, p->fm, p->lam, &iters, &outer);
      if (status != SSO_OK && status != SSO_ENOTCONV) return status;
      lam = p->lam;
    }
  } else if (kind == SSO_OBJ_LINEAR || kind == SSO_OBJ_USER) {
    if (!dg_du) return SSO_EINVAL;
    c_u = 0.0;
    TRY_HIP(launch_mask_vector(p->m, dg_du, p->rhs, s));
    int outer = 0;
    status = run_solver(p, p->rhs, p->lam, &iters, &outer);
    if (status != SSO_OK && status != SSO_ENOTCONV) return status;
    lam = p->lam;
  } else {
    return SSO_EINVAL;
  }
  TRY_HIP(launch_adjoint_terms(p->m, p->pat, p->u, lam, c_lam, c_u, p->gbeam, p->gquad, s));
  TRY_HIP(launch_gather(p->m, p->pat, p->gbeam, p->gquad, dg_dxyz, dg_dt, dg_dscale, s));
  TRY_HIP(hipEventRecord(p->ev[5], s));
  TRY_HIP(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = iters;
    stats->t_adj_us = elapsed_us(p->ev[4], p->ev[5]);
    stats->bytes_moved = solve_bytes(p, iters, 0, true);
  }
  return status;
}

int sso_size_objective(sso_problem* p, double eps1, double u_max, double t_min,
                       double* out_host, double* dg_dxyz, double* dg_dt, sso_stats* stats) {
  if (!size_args_ok(p, eps1, u_max, t_min, out_host, dg_dxyz)) return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  if (!p->xpart) {
    TRY_HIP(dev_alloc(&p->xpart, 2 * SIZE_XWG, p->s));
    TRY_HIP(dev_alloc(&p->gw, 14 * (int64_t)p->m.n_quads, p->s));
    TRY_HIP(dev_alloc(&p->wv, p->m.n_quads, p->s));
  }
  return size_objective_impl(p, eps1, u_max, t_min, out_host, dg_dxyz, dg_dt, stats,
                             p->xpart, p->gw, p->wv);
}

int sso_size_penalty_update(double eps1, int violated, double kappa, double* eps1_next) {
  if (!eps1_next || !(eps1 >= 0.0) || !std::isfinite(eps1) || !(kappa > 0.0) ||
      !std::isfinite(kappa))
    return SSO_EINVAL;
  *eps1_next = violated ? eps1 * kappa : eps1 / kappa;
  return SSO_OK;
}

int sso_size_objective_noalloc(sso_problem* p, double eps1, double u_max, double t_min,
                               double* out_host, double* dg_dxyz, double* dg_dt,
                               sso_stats* stats) {
  if (p && p->m.n_quads > SSO_NOALLOC_MAX_QUADS) return SSO_ESIZE;
  if (!size_args_ok(p, eps1, u_max, t_min, out_host, dg_dxyz)) return SSO_EINVAL;
  double* base = nullptr;
  const int st = scratch_address(p->device, &base);
  if (st != SSO_OK) return st;
  // partials, then the per-quad volume terms and shares; every entry is written before it is
  // read, so nothing needs clearing between calls
  double* xpart = base;
  double* gw = xpart + 2 * SIZE_XWG;
  double* wv = gw + 14 * (int64_t)p->m.n_quads;
  return size_objective_impl(p, eps1, u_max, t_min, out_host, dg_dxyz, dg_dt, stats, xpart, gw,
                             wv);
}

int sso_hat_filter(sso_problem* p, int32_t n, const int32_t* nodes, const double* g,
                   double radius, double* out) {
  if (!p || n < 0 || (n > 0 && (!g || !out)) || !(radius > 0.0) || !std::isfinite(radius))
    return SSO_EINVAL;
  if (!nodes && n > p->m.n_nodes) return SSO_EINVAL;
  hipStream_t s = p->s;
  TRY_HIP(hipMemsetAsync(p->d_err, 0, sizeof(unsigned), s));
  TRY_HIP(launch_hat_filter(n, nodes, p->m, g, radius, out, p->d_err, s));
  return read_errors(p);
}

int sso_pattern(sso_problem* p, const int32_t** row_ptr, const int32_t** col,
                const int32_t** perm, const int32_t** seg, int64_t* nnz, int64_t* n_coo) {
  if (!p) return SSO_EINVAL;
  if (p->n_coo >= ((int64_t)1 << 31) || 36 * p->pat.n_blocks >= ((int64_t)1 << 31))
    return SSO_EINVAL;
  AllocScope ac(&p->bytes, &p->mem);
  const int64_t nz = 36 * p->pat.n_blocks;
  hipStream_t s = p->s;
  if (!p->row_ptr) {
    TRY_HIP(dev_alloc(&p->row_ptr, 6 * (int64_t)p->m.n_nodes + 1, s));
    TRY_HIP(dev_alloc(&p->col, nz, s));
    TRY_HIP(dev_alloc(&p->perm, p->n_coo, s));
    TRY_HIP(dev_alloc(&p->seg, nz + 1, s));
    TRY_HIP(build_scalar_view(p->m, p->pat, p->row_ptr, p->col, p->perm, p->seg, p->s));
    TRY_HIP(hipStreamSynchronize(p->s));
  }
  if (row_ptr) *row_ptr = p->row_ptr;
  if (col) *col = p->col;
  if (perm) *perm = p->perm;
  if (seg) *seg = p->seg;
  if (nnz) *nnz = nz;
  if (n_coo) *n_coo = p->n_coo;
  return SSO_OK;
}

int sso_matrix(sso_problem* p, double* vals, double* f) {
  if (!p || !vals) return SSO_EINVAL;
  TRY_HIP(launch_scalar_values(p->m, p->pat, p->K, vals, p->s));
  if (f)
    TRY_HIP(hipMemcpyAsync(f, p->f, sizeof(double) * 6 * (size_t)p->m.n_nodes,
                           hipMemcpyDeviceToDevice, p->s));
  TRY_HIP(hipStreamSynchronize(p->s));
  return SSO_OK;
}

int sso_problem_bytes(const sso_problem* p, int64_t* bytes) {
  if (!p || !bytes) return SSO_EINVAL;
  *bytes = p->bytes;
  return SSO_OK;
}

int sso_sizes(const sso_problem* p, int64_t* n_dof, int64_t* n_blocks, int64_t* nnz) {
  if (!p) return SSO_EINVAL;
  if (n_dof) *n_dof = 6 * (int64_t)p->m.n_nodes;
  if (n_blocks) *n_blocks = p->pat.n_blocks;
  if (nnz) *nnz = 36 * p->pat.n_blocks;
  return SSO_OK;
}

const char* sso_strerror(int status) {
  switch (status) {
    case SSO_OK: return "ok";
    case SSO_EINVAL: return "invalid argument or degenerate element";
    case SSO_ENOMEM: return "device memory allocation failed";
    case SSO_EHIP: return "HIP runtime error";
    case SSO_ENOTCONV: return "PCG did not reach the residual target within max_it";
    case SSO_EBREAKDOWN: return "PCG breakdown: stiffness not positive definite";
    case SSO_ESIZE: return "problem larger than the static scratch of the no-allocation entry point";
    default: return "unknown status";
  }
}

void sso_problem_destroy(sso_problem* p) { free_problem(p); }

int sso_pool_trim(int device, uint64_t keep_bytes) {
  if (device < 0 || device >= MAX_DEVICES) return SSO_EINVAL;
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(pool_mutex);
    pool = pools[device];
  }
  if (!pool) return SSO_OK;
  TRY_HIP(hipMemPoolTrimTo(pool, (size_t)keep_bytes));
  return SSO_OK;
}

}  // extern "C"
