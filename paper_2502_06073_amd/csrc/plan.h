// Compile-time plan of the equivariant layers: which channelwise tensor
// products exist in each layer, where their operands live and where their
// results go.  Used by host code (weight layout, workspace sizes) and by the
// kernels (fully unrolled tensor-product loops with constant indices).
//
// Tensor features carry irreps (l, p) with l <= l_max and parity p = +-1
// ("l = 2 in full O(3) symmetry", Methodology / Model Training).  The first
// layer's input features come from spherical harmonics and have the natural
// parity (-1)^l.  A path ((l1,p1), l2 -> (l3,p3)) combines an edge feature of
// irrep (l1,p1) with the environment sum's degree l2 (parity (-1)^l2) into
// degree l3 with |l1-l2| <= l3 <= min(l1+l2, l_max) and p3 = p1 (-1)^l2.  The
// last layer only produces (0,+) scalars.  Paths whose outputs no later step
// reads are pruned (they cannot change the energy).  Paths are ordered by
// (l1, p1 [+ first], l2, l3, p3 [+ first]); irreps by (l, p [+ first]).
#pragma once
#include <stdint.h>

namespace afm {

constexpr int kMaxLmax = 3;
constexpr int kMaxLayers = 4;
constexpr int kMaxPaths = 40;   // l_max = 3 in full O(3): 34 in a hidden layer
constexpr int kMaxIrreps = 8;
constexpr int kMaxComps = 32;   // sum of (2l+1) over the irreps of one layer

struct Irrep {
  int l = 0, p = 1;
};

struct PathT {
  int l1 = 0, p1 = 1, l2 = 0, l3 = 0, p3 = 1;
  int in_off = 0;    // component offset of (l1,p1) in the input features
  int out_off = -1;  // component offset of (l3,p3) in the output features (-1: none)
  int s_idx = -1;    // index among the layer's (0,+) paths (-1: not a scalar path)
};

struct LayerPlan {
  int n_paths = 0;
  PathT p[kMaxPaths] = {};
  int n_in = 0;
  Irrep in[kMaxIrreps] = {};
  int in_off[kMaxIrreps] = {};
  int n_in_comps = 0;
  int n_out = 0;
  Irrep out[kMaxIrreps] = {};
  int out_off[kMaxIrreps] = {};
  int n_out_comps = 0;
  int n0e = 0;       // number of (0,+) paths = scalars per channel fed to the MLP
};

struct Plan {
  int lmax = 0, n_layers = 0;
  bool ok = false;
  LayerPlan layer[kMaxLayers] = {};
};

constexpr int pkey(int p) { return p == 1 ? 0 : 1; }
constexpr int irrep_rank(int l, int p) { return 2 * l + pkey(p); }
constexpr int ipow_m1(int l) { return (l & 1) ? -1 : 1; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int iabs(int a) { return a < 0 ? -a : a; }

constexpr bool path_less(const PathT& a, const PathT& b) {
  if (a.l1 != b.l1) return a.l1 < b.l1;
  if (a.p1 != b.p1) return pkey(a.p1) < pkey(b.p1);
  if (a.l2 != b.l2) return a.l2 < b.l2;
  if (a.l3 != b.l3) return a.l3 < b.l3;
  return pkey(a.p3) < pkey(b.p3);
}

// irreps present in a bitmask over irrep_rank, in canonical order
constexpr int fill_irreps(unsigned mask, Irrep* out, int* off) {
  int n = 0, o = 0;
  for (int r = 0; r < 2 * (kMaxLmax + 1); ++r) {
    if (mask & (1u << r)) {
      out[n].l = r / 2;
      out[n].p = (r & 1) ? -1 : 1;
      off[n] = o;
      o += 2 * out[n].l + 1;
      ++n;
    }
  }
  return n;
}

constexpr Plan make_plan(int lmax, int n_layers) {
  Plan P{};
  P.lmax = lmax;
  P.n_layers = n_layers;
  if (lmax < 0 || lmax > kMaxLmax || n_layers < 1 || n_layers > kMaxLayers) return P;
  // forward availability with every output kept (last layer: only 0e)
  unsigned avail[kMaxLayers + 1] = {};
  for (int l = 0; l <= lmax; ++l) avail[0] |= 1u << irrep_rank(l, ipow_m1(l));
  PathT full[kMaxLayers][40] = {};
  int nfull[kMaxLayers] = {};
  for (int L = 1; L <= n_layers; ++L) {
    int n = 0;
    for (int r = 0; r < 2 * (lmax + 1); ++r) {
      if (!(avail[L - 1] & (1u << r))) continue;
      int l1 = r / 2, p1 = (r & 1) ? -1 : 1;
      for (int l2 = 0; l2 <= lmax; ++l2)
        for (int l3 = iabs(l1 - l2); l3 <= imin(l1 + l2, lmax); ++l3) {
          int p3 = p1 * ipow_m1(l2);
          if (L == n_layers && !(l3 == 0 && p3 == 1)) continue;
          PathT t{};
          t.l1 = l1; t.p1 = p1; t.l2 = l2; t.l3 = l3; t.p3 = p3;
          full[L - 1][n++] = t;
          avail[L] |= 1u << irrep_rank(l3, p3);
        }
    }
    nfull[L - 1] = n;
  }
  // backward pruning: keep outputs read by the next layer, or 0e scalars
  for (int L = n_layers - 1; L >= 1; --L) {
    unsigned used = 0;
    for (int k = 0; k < nfull[L]; ++k) used |= 1u << irrep_rank(full[L][k].l1, full[L][k].p1);
    int n = 0;
    for (int k = 0; k < nfull[L - 1]; ++k) {
      const PathT t = full[L - 1][k];
      if ((used & (1u << irrep_rank(t.l3, t.p3))) || (t.l3 == 0 && t.p3 == 1))
        full[L - 1][n++] = t;
    }
    nfull[L - 1] = n;
  }
  // sort, then fill offsets
  for (int L = 0; L < n_layers; ++L) {
    for (int a = 1; a < nfull[L]; ++a)
      for (int b = a; b > 0 && path_less(full[L][b], full[L][b - 1]); --b) {
        PathT tmp = full[L][b];
        full[L][b] = full[L][b - 1];
        full[L][b - 1] = tmp;
      }
  }
  unsigned in_mask = avail[0];
  for (int L = 0; L < n_layers; ++L) {
    LayerPlan& lp = P.layer[L];
    unsigned out_mask = 0;
    if (L + 1 < n_layers)
      for (int k = 0; k < nfull[L]; ++k) out_mask |= 1u << irrep_rank(full[L][k].l3, full[L][k].p3);
    lp.n_in = fill_irreps(in_mask, lp.in, lp.in_off);
    lp.n_in_comps = 0;
    for (int k = 0; k < lp.n_in; ++k) lp.n_in_comps += 2 * lp.in[k].l + 1;
    lp.n_out = fill_irreps(out_mask, lp.out, lp.out_off);
    lp.n_out_comps = 0;
    for (int k = 0; k < lp.n_out; ++k) lp.n_out_comps += 2 * lp.out[k].l + 1;
    lp.n_paths = nfull[L];
    int s = 0;
    for (int k = 0; k < nfull[L]; ++k) {
      PathT t = full[L][k];
      for (int q = 0; q < lp.n_in; ++q)
        if (lp.in[q].l == t.l1 && lp.in[q].p == t.p1) t.in_off = lp.in_off[q];
      t.out_off = -1;
      for (int q = 0; q < lp.n_out; ++q)
        if (lp.out[q].l == t.l3 && lp.out[q].p == t.p3) t.out_off = lp.out_off[q];
      t.s_idx = (t.l3 == 0 && t.p3 == 1) ? s++ : -1;
      lp.p[k] = t;
    }
    lp.n0e = s;
    in_mask = out_mask;
  }
  P.ok = true;
  return P;
}

// Dense mixing: per-edge products T of every path of a layer, path after
// path (2 l3 + 1 components each); offset of path k and the total.
constexpr int dense_t_off(const LayerPlan& lp, int k) {
  int o = 0;
  for (int q = 0; q < k; ++q) o += 2 * lp.p[q].l3 + 1;
  return o;
}
constexpr int dense_t_comps(const LayerPlan& lp) { return dense_t_off(lp, lp.n_paths); }

template <int LMAX, int NL>
struct PlanCT {
  static constexpr Plan plan = make_plan(LMAX, NL);
  static_assert(plan.ok, "unsupported (l_max, n_layers)");
};

}  // namespace afm
