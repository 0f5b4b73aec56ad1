// Native host checks of libhipsso, built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host code (tests/test_native_host.py builds and runs it on the CPU; no GPU is touched):
//   * every C-ABI entry point on its argument-error paths, which return before any device work;
//   * the host-only entry points (sso_strerror, sso_size_penalty_update);
//   * the pattern checker of the debug mode (check_pattern) on block patterns built here from the
//     element lists by a plain map, and on copies of them with one invariant broken each.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include "hipsso.h"
#include "sso_internal.h"

static int failures = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);         \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static void abi_argument_paths() {
  sso_problem* p = nullptr;
  sso_mesh m;
  std::memset(&m, 0, sizeof m);
  CHECK(sso_problem_create(nullptr, nullptr, nullptr, &p) == SSO_EINVAL);
  CHECK(sso_problem_create(&m, nullptr, nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL && p == nullptr);  // 0 nodes
  double xyz[12] = {};
  uint8_t fixed[24] = {};
  double f[24] = {};
  int32_t conn[4] = {0, 1, 2, 3};
  double prop[6] = {};
  m.n_nodes = 4;
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL);   // no coordinates
  m.xyz = xyz;
  m.fixed = fixed;
  m.f_nodal = f;
  m.n_beams = -1;
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL);
  m.n_beams = 1;
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL);   // no member arrays
  m.n_beams = 0;
  m.n_quads = 1;
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL);   // no quad arrays
  m.quad_nodes = conn;
  m.quad_prop = prop;
  m.n_quads = 1 << 28;                                                 // 16 n_quads >= 2^31
  CHECK(sso_problem_create(&m, nullptr, nullptr, &p) == SSO_EINVAL);
  m.n_quads = 1;
  sso_options bad[7];
  for (auto& o : bad) {
    o.precision = SSO_PREC_FP64;
    o.rtol = 1e-8;
    o.max_it = 100;
    o.refine_steps = 2;
    o.profile_every = 0;
    o.inner_rtol = 0.0;
    o.solver = SSO_SOLVER_AUTO;
    o.inner_max_it = 0;
  }
  bad[0].precision = 7;
  bad[1].rtol = -1.0;
  bad[2].max_it = 0;
  bad[3].inner_rtol = 1.0;
  bad[4].solver = 9;
  bad[5].inner_max_it = -3;
  bad[6].solver = SSO_SOLVER_WG;      // the one-workgroup solver runs in FP64 only
  bad[6].precision = SSO_PREC_MIXED;
  for (auto& o : bad) CHECK(sso_problem_create(&m, &o, nullptr, &p) == SSO_EINVAL && !p);
  CHECK(sso_problem_update(nullptr, nullptr, nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_set_options(nullptr, &bad[0]) == SSO_EINVAL);
  CHECK(sso_solve(nullptr, nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_solve_begin(nullptr) == SSO_EINVAL);
  CHECK(sso_solve_end(nullptr, nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_batch_create(nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_batch_iterate(nullptr, nullptr, 0, 1, nullptr) == SSO_EINVAL);
  double g = 0.0, out3[3] = {};
  CHECK(sso_objective(nullptr, SSO_OBJ_COMPLIANCE, nullptr, &g) == SSO_EINVAL);
  CHECK(sso_adjoint(nullptr, SSO_OBJ_COMPLIANCE, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        SSO_EINVAL);
  CHECK(sso_size_objective(nullptr, 1.0, 1.0, 1.0, out3, nullptr, nullptr, nullptr) ==
        SSO_EINVAL);
  CHECK(sso_size_objective_noalloc(nullptr, 1.0, 1.0, 1.0, out3, nullptr, nullptr, nullptr) ==
        SSO_EINVAL);
  CHECK(sso_hat_filter(nullptr, 3, nullptr, nullptr, 1.0, nullptr) == SSO_EINVAL);
  const int32_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
  int64_t i0 = 0, i1 = 0, i2 = 0;
  CHECK(sso_pattern(nullptr, &a0, &a1, &a2, &a3, &i0, &i1) == SSO_EINVAL);
  CHECK(sso_matrix(nullptr, nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_sizes(nullptr, &i0, &i1, &i2) == SSO_EINVAL);
  CHECK(sso_problem_bytes(nullptr, &i0) == SSO_EINVAL);
  CHECK(sso_batch_launch(nullptr, nullptr, 0, 1) == SSO_EINVAL);
  CHECK(sso_batch_wait(nullptr, nullptr, 0, nullptr) == SSO_EINVAL);
  CHECK(sso_problem_set_stream(nullptr, nullptr) == SSO_EINVAL);
  CHECK(sso_pool_trim(-1, 0) == SSO_EINVAL);
  CHECK(sso_pool_trim(1 << 20, 0) == SSO_EINVAL);
  CHECK(sso_pool_trim(0, 0) == SSO_OK);   // no pool was ever created: nothing to release
  for (int k = -10; k <= 5; ++k) CHECK(sso_strerror(k) && std::strlen(sso_strerror(k)) > 0);
  sso_problem_destroy(nullptr);
  sso_batch_destroy(nullptr);
  double e = 0.0;
  CHECK(sso_size_penalty_update(2.0, 1, 1.015, &e) == SSO_OK && e == 2.0 * 1.015);
  CHECK(sso_size_penalty_update(2.0, 0, 1.015, &e) == SSO_OK && e == 2.0 / 1.015);
  CHECK(sso_size_penalty_update(-1.0, 0, 1.015, &e) == SSO_EINVAL);
  CHECK(sso_size_penalty_update(1.0, 0, 0.0, &e) == SSO_EINVAL);
  CHECK(sso_size_penalty_update(NAN, 0, 1.015, &e) == SSO_EINVAL);
  CHECK(sso_size_penalty_update(1.0, 0, INFINITY, &e) == SSO_EINVAL);
  CHECK(sso_size_penalty_update(1.0, 0, 1.015, nullptr) == SSO_EINVAL);
}

// A block pattern built from the element lists with an ordered map (the reference for the
// checker's own tests): slot (I, J) holds the ids of its block contributions in ascending order.
struct Built {
  int n_nodes, n_beams, n_quads;
  std::vector<int32_t> beams, quads, brow, bcol, bseg, bperm, bslot, bdiag, bsrow, est, ell,
      sym;
  int ell_w = 0;
  sso::HostPattern view() const {
    sso::HostPattern h;
    h.n_nodes = n_nodes;
    h.n_beams = n_beams;
    h.n_quads = n_quads;
    h.ell_w = ell_w;
    h.n_blocks = (int64_t)bcol.size();
    h.n_bcoo = (int64_t)bperm.size();
    h.brow_ptr = brow.data();
    h.bcol = bcol.data();
    h.bseg = bseg.data();
    h.bperm = bperm.data();
    h.bslot = bslot.data();
    h.bdiag = bdiag.data();
    h.bsrow = bsrow.data();
    h.estart = est.data();
    h.bcol_ell = ell.data();
    h.beam_nodes = beams.data();
    h.quad_nodes = quads.data();
    h.bsym = sym.data();
    return h;
  }
};

static Built build(int n_nodes, const std::vector<int32_t>& beams,
                   const std::vector<int32_t>& quads) {
  Built b;
  b.n_nodes = n_nodes;
  b.n_beams = (int)beams.size() / 2;
  b.n_quads = (int)quads.size() / 4;
  b.beams = beams;
  b.quads = quads;
  std::map<std::pair<int, int>, std::vector<int32_t>> slots;
  for (int I = 0; I < n_nodes; ++I) slots[{I, I}];
  int32_t id = 0;
  for (int e = 0; e < b.n_beams; ++e)
    for (int la = 0; la < 2; ++la)
      for (int lb = 0; lb < 2; ++lb) slots[{beams[2 * e + la], beams[2 * e + lb]}].push_back(id++);
  for (int e = 0; e < b.n_quads; ++e)
    for (int la = 0; la < 4; ++la)
      for (int lb = 0; lb < 4; ++lb) slots[{quads[4 * e + la], quads[4 * e + lb]}].push_back(id++);
  b.brow.assign(n_nodes + 1, 0);
  b.est.assign(n_nodes + 1, 0);
  b.bdiag.assign(n_nodes, -1);
  b.bperm.reserve(id);
  b.bseg.push_back(0);
  int max_row = 0;
  for (const auto& kv : slots) {
    const int I = kv.first.first, J = kv.first.second;
    const int32_t s = (int32_t)b.bcol.size();
    b.bcol.push_back(J);
    b.bsrow.push_back(I);
    if (I == J) b.bdiag[I] = s;
    for (int32_t j : kv.second) {
      b.bperm.push_back(j);
      b.bslot.push_back(s);
    }
    b.bseg.push_back((int32_t)b.bperm.size());
    b.brow[I + 1] = s + 1;
  }
  for (int I = 0; I < n_nodes; ++I) {
    if (b.brow[I + 1] < b.brow[I]) b.brow[I + 1] = b.brow[I];
    const int cnt = b.brow[I + 1] - b.brow[I];
    if (cnt > max_row) max_row = cnt;
  }
  for (int I = 0; I <= n_nodes; ++I) b.est[I] = I < n_nodes ? b.bseg[b.brow[I]] : id;
  std::map<std::pair<int, int>, int32_t> slot_of;
  for (size_t s = 0; s < b.bcol.size(); ++s) slot_of[{b.bsrow[s], b.bcol[s]}] = (int32_t)s;
  for (size_t s = 0; s < b.bcol.size(); ++s) {
    b.sym.push_back(b.bcol[s]);
    b.sym.push_back(b.bcol[s] < b.bsrow[s] ? slot_of.at({b.bcol[s], b.bsrow[s]}) : (int32_t)s);
  }
  b.ell_w = sso::ell_width(max_row);
  b.ell.assign((size_t)n_nodes * (b.ell_w > 0 ? b.ell_w : 0), 0);
  for (int I = 0; I < n_nodes && b.ell_w > 0; ++I)
    for (int u = 0; u < b.ell_w; ++u)
      b.ell[(size_t)I * b.ell_w + u] =
          u < b.brow[I + 1] - b.brow[I] ? b.bcol[b.brow[I] + u] : I;
  return b;
}

static int check(const Built& b) {
  char msg[256];
  return sso::check_pattern(b.view(), msg, sizeof msg);
}

static void pattern_checks() {
  // a 3 x 3 quad grid (16 nodes) with two members, and an isolated node 16
  std::vector<int32_t> quads;
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) {
      const int a = 4 * j + i;
      quads.insert(quads.end(), {a, a + 1, a + 5, a + 4});
    }
  const std::vector<int32_t> beams = {0, 15, 5, 10};
  const Built b = build(17, beams, quads);
  CHECK(b.ell_w == 9 || b.ell_w == 12);
  CHECK(check(b) == 0);
  const Built g = build(6, {0, 1, 1, 2, 2, 3, 3, 4, 4, 5}, {});
  CHECK(check(g) == 0);
  // one broken invariant at a time, each caught by its own check
  {
    Built c = b;
    c.brow[17] -= 1;
    CHECK(check(c) == 1);
  }
  {
    Built c = b;
    std::swap(c.bcol[c.brow[5]], c.bcol[c.brow[5] + 1]);
    CHECK(check(c) == 2);
  }
  {
    Built c = b;
    c.bcol[3] = 99;
    CHECK(check(c) == 2);
  }
  {
    Built c = b;
    c.bdiag[5] = c.brow[5];
    CHECK(check(c) == 3);
  }
  {
    Built c = b;
    c.bseg[4] = c.bseg[5] + 1;
    CHECK(check(c) == 4);
  }
  {
    Built c = b;
    c.bperm[7] = c.bperm[8];
    CHECK(check(c) == 5);
  }
  {
    Built c = b;
    const int32_t s = c.brow[6];
    std::swap(c.bperm[c.bseg[s]], c.bperm[c.bseg[s + 3]]);   // a contribution in another slot
    CHECK(check(c) == 6);
  }
  {
    Built c = b;
    c.est[6] += 1;
    CHECK(check(c) == 7);
  }
  {
    Built c = b;
    c.ell[(size_t)16 * c.ell_w + c.ell_w - 1] = 3;             // padding of the isolated node
    CHECK(check(c) == 8);
  }
  {
    Built c = b;
    const int32_t s = c.brow[5];                               // (5, 0): left of the diagonal
    c.sym[2 * s + 1] = c.sym[2 * s + 3];
    CHECK(check(c) == 9);
  }
  {
    Built c = b;
    const int32_t s = c.brow[5] + 5;                           // right of the diagonal: itself
    c.sym[2 * s + 1] = c.sym[2 * c.brow[5] + 1];
    CHECK(check(c) == 9);
  }
  {
    Built c = b;
    c.sym[2 * c.bdiag[16] + 1] = c.bdiag[15];                 // a diagonal names another row's
    CHECK(check(c) == 9);
  }
  {
    Built c = b;
    c.sym[2 * c.brow[9]] = c.bcol[c.brow[9] + 1];              // a wrong column
    CHECK(check(c) == 9);
  }
}

int main() {
  abi_argument_paths();
  pattern_checks();
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
