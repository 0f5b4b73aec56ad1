// Host-side consistency checks of the block pattern, the sort permutation and the padded block
// rows (debug mode: HIPSSO_DEBUG set at sso_problem_create; and the native host tests).
//
// The pattern of Sec. 2.2.1's sparse K is built on the GPU (pattern.hip); these checks restate
// what it must satisfy, element by element, in plain loops:
//   1 brow_ptr: 0 at the start, n_blocks at the end, strictly increasing (every row holds its
//     diagonal block);
//   2 bcol: within [0, n_nodes), strictly increasing along each row;
//   3 bdiag / bsrow: the diagonal slot of row I holds column I; every slot knows its row;
//   4 bseg: 0 at the start, n_bcoo at the end, each slot's segment non-empty except for an
//     isolated node's diagonal, non-decreasing;
//   5 bperm: a permutation of the block contribution ids; bslot: the slot of each position;
//   6 every contribution sits in the slot of its own (row node, column node), ids ascending
//     within a slot (the stable order of the element-major contribution list);
//   7 estart: each row's first sorted position;
//   8 padded rows (ell_w > 0): each row's columns in order, then the row's own node;
//   9 bsym: each slot's column, then its value slot: the slot of (J, I) for a block (I, J) with
//     J < I (the pattern is structurally symmetric: an element couples its nodes both ways),
//     the slot itself for J >= I.
#include <cstdio>
#include <vector>

#include "sso_internal.h"

namespace sso {

namespace {

int fail(char* msg, size_t len, int code, const char* what, int64_t at) {
  if (msg && len) std::snprintf(msg, len, "pattern check %d failed: %s (at %lld)", code, what,
                                (long long)at);
  return code;
}

}  // namespace

int check_pattern(const HostPattern& h, char* msg, size_t len) {
  const int n = h.n_nodes;
  const int64_t nb = h.n_blocks, nc = h.n_bcoo;
  if (n <= 0 || nb < n || nc < 0) return fail(msg, len, 1, "sizes", 0);
  if (h.brow_ptr[0] != 0 || h.brow_ptr[n] != nb) return fail(msg, len, 1, "brow_ptr ends", n);
  for (int I = 0; I < n; ++I)
    if (h.brow_ptr[I + 1] <= h.brow_ptr[I]) return fail(msg, len, 1, "brow_ptr order", I);
  for (int I = 0; I < n; ++I)
    for (int32_t s = h.brow_ptr[I]; s < h.brow_ptr[I + 1]; ++s) {
      if (h.bcol[s] < 0 || h.bcol[s] >= n) return fail(msg, len, 2, "bcol range", s);
      if (s > h.brow_ptr[I] && h.bcol[s] <= h.bcol[s - 1])
        return fail(msg, len, 2, "bcol order", s);
      if (h.bsrow[s] != I) return fail(msg, len, 3, "bsrow", s);
    }
  for (int I = 0; I < n; ++I) {
    const int32_t d = h.bdiag[I];
    if (d < h.brow_ptr[I] || d >= h.brow_ptr[I + 1] || h.bcol[d] != I)
      return fail(msg, len, 3, "bdiag", I);
  }
  if (h.bseg[0] != 0 || h.bseg[nb] != nc) return fail(msg, len, 4, "bseg ends", nb);
  for (int64_t s = 0; s < nb; ++s) {
    if (h.bseg[s + 1] < h.bseg[s]) return fail(msg, len, 4, "bseg order", s);
    if (h.bseg[s + 1] == h.bseg[s] && h.bcol[s] != h.bsrow[s])
      return fail(msg, len, 4, "empty off-diagonal slot", s);
  }
  std::vector<char> seen(nc > 0 ? nc : 1, 0);
  for (int64_t k = 0; k < nc; ++k) {
    const int32_t j = h.bperm[k];
    if (j < 0 || j >= nc || seen[j]) return fail(msg, len, 5, "bperm not a permutation", k);
    seen[j] = 1;
  }
  for (int64_t s = 0; s < nb; ++s)
    for (int32_t k = h.bseg[s]; k < h.bseg[s + 1]; ++k) {
      if (h.bslot[k] != s) return fail(msg, len, 5, "bslot", k);
      const BlockRef r = decode_block(h.bperm[k], h.n_beams);
      const int32_t* conn = r.quad ? h.quad_nodes + 4 * (int64_t)r.e : h.beam_nodes + 2 * (int64_t)r.e;
      if ((r.quad ? r.e >= h.n_quads : r.e >= h.n_beams) || conn[r.la] != h.bsrow[s] ||
          conn[r.lb] != h.bcol[s])
        return fail(msg, len, 6, "contribution in a foreign slot", k);
      if (k > h.bseg[s] && h.bperm[k] <= h.bperm[k - 1])
        return fail(msg, len, 6, "ids not ascending in a slot", k);
    }
  for (int I = 0; I < n; ++I)
    if (h.estart[I] != h.bseg[h.brow_ptr[I]]) return fail(msg, len, 7, "estart", I);
  if (h.estart[n] != nc) return fail(msg, len, 7, "estart end", n);
  if (h.ell_w > 0) {
    for (int I = 0; I < n; ++I) {
      const int32_t rb = h.brow_ptr[I], cnt = h.brow_ptr[I + 1] - rb;
      if (cnt > h.ell_w) return fail(msg, len, 8, "row wider than the padded width", I);
      for (int u = 0; u < h.ell_w; ++u) {
        const int32_t want = u < cnt ? h.bcol[rb + u] : I;
        if (h.bcol_ell[(int64_t)I * h.ell_w + u] != want)
          return fail(msg, len, 8, "padded row", (int64_t)I * h.ell_w + u);
      }
    }
  }
  for (int64_t s = 0; s < nb; ++s) {
    const int32_t J = h.bsym[2 * s], m = h.bsym[2 * s + 1];
    const bool ok = J == h.bcol[s] &&
                    (J >= h.bsrow[s] ? m == s
                                     : m >= 0 && m < nb && h.bsrow[m] == J && h.bcol[m] == h.bsrow[s]);
    if (!ok) return fail(msg, len, 9, "bsym", s);
  }
  return 0;
}

}  // namespace sso
