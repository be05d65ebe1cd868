// BF16 MFMA chains for the per-edge MLPs (gfx950, v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): the two-body MLP, the linear environment embeddings and
// the latent MLPs with their residual updates (Methodology / Model Training:
// two-body latent MLP, "embedding MLP ... linear projection", latent MLP,
// SiLU), forward and adjoint.
//
// Mapping.  A workgroup owns a tile of 64 edges with 8 wavefronts, or of
// 128 edges with 16 (the edge-tile shape, a property of the model; the
// kernels of both shapes are instantiated from mfma_chain_tile.h).  Each
// wavefront covers 4 column blocks of 16 edges.  Each layer is computed
// transposed, Y^T = W X^T: the weights are the MFMA A operand (16 output
// features x 32 input features per fragment), the edges the B/C columns.
// The tile's activations live in LDS as bf16 B fragments (two ping-pong
// buffers), written once by the wavefront that computed them and read by
// all; each wavefront owns pairs of 16-row output blocks and streams its
// own weight fragments from L2 into registers, so a weight byte is fetched
// once per 64 edges and an LDS fragment feeds 2 x (rows per wavefront)
// MFMAs.  One barrier per layer.
// A C block's lane group g holds output features 4g..4g+3, so the pair of
// blocks (2p, 2p+1) packs into the B fragment of k-block p of the next layer
// when input k-slot (g, i) carries feature
//   phi(kb, g, i) = 32 kb + 4 g + (i & 3) + 16 (i >> 2);
// every weight fragment is packed on the host with the same permutation
// (MFMA pairs A and B k-slots identically, so the product is unchanged).
// Every weight is held as an unevaluated sum of two bf16 numbers (hi + lo,
// lo = bf16(w - hi)) and each fragment product is issued as two MFMAs into
// the same FP32 accumulator, so the weights keep ~16 mantissa bits while
// activations are rounded to bf16 once per layer.  Rounding the weights
// alone would perturb the model itself, an error common to every edge that
// does not average out over a structure; activation rounding is independent
// per edge -- except where near-equal activations make it correlated: the
// two-body MLP's hidden activations are also carried as two bf16 terms.
// Pre-activations are stored as bf16 in a tile-native layout read back by
// the adjoint.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "device_util.h"
#include "edge_layout.h"
#include "internal.h"

namespace afm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSplit = 2;         // bf16 terms per weight (hi, lo)
// The adjoint chains (forces) use the same terms as the forward, so that the
// forces are the gradient of the reported energy up to the bf16 rounding of
// activations and gradients.  The fast-adjoint variant uses the hi term
// alone there: rounding a weight to bf16 shifts every edge energy the same
// way (the energy keeps lo to stay within 1 meV/atom), while in the adjoint
// it adds a force error of the size the bf16 activations already cause
// (emulated in FP64 on a 125-atom lattice: 3.9 -> 5.1 meV/A RMS, bound
// 20 meV/A) and halves the adjoint's weight stream and MFMAs -- at the price
// of forces that belong to a model ~4 meV/atom away from the reported one.
// The environment embeddings omega = W_env x use the hi term alone in the
// forward as well: omega enters the energy only through the per-atom sums
// and tensor products, and rounding W_env to bf16 moved the emulated
// energy by 0.04 meV/atom (the two-body and latent weights, 2.2 and 1.8).
constexpr int kSplitEnv = 1;

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// host packing

static uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// M(r, k) = transpose ? W[k * R + r] : W[r * K + k]; fragments
// [RB][KB][2][64][8] with the hi part of the weight pairs first, lo second;
// RB is rounded up to an even count (zero rows)
static void pack_matrix(const double* W, int R, int K, bool transpose, std::vector<char>& out,
                        int64_t* off) {
  const int RB = 2 * cdiv(R, 32), KB = cdiv(K, 32);   // row blocks padded to whole pairs
  int64_t o = (int64_t)out.size();
  o = (o + 255) & ~int64_t(255);
  out.resize(o + (int64_t)RB * KB * kSplit * 64 * 16, 0);
  uint16_t* p = reinterpret_cast<uint16_t*>(out.data() + o);
  for (int rb = 0; rb < RB; ++rb)
    for (int kb = 0; kb < KB; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = 16 * rb + (lane & 15), g = lane >> 4;
        for (int i = 0; i < 8; ++i) {
          const int k = 32 * kb + 4 * g + (i & 3) + 16 * (i >> 2);
          double v = 0.0;
          if (r < R && k < K) v = transpose ? W[(int64_t)k * R + r] : W[(int64_t)r * K + k];
          const uint16_t hi = bf16_rne((float)v);
          const uint16_t lo = bf16_rne((float)(v - bf16_value(hi)));
          const int64_t base = (((int64_t)rb * KB + kb) * kSplit * 64 + lane) * 8 + i;
          p[base] = hi;
          p[base + 64 * 8] = lo;
        }
      }
  *off = o;
}

static const afm_param_block* blk(const afm_model* m, const char* name) {
  for (auto& b : m->blocks)
    if (strcmp(b.name, name) == 0) return &b;
  return nullptr;
}

struct FragOffsets {
  int64_t tbf[kMaxTwobody], tbb[kMaxTwobody];
  int64_t envf[kMaxLayers], envb[kMaxLayers];
  int64_t latf[kMaxLayers][kMaxDepth], latb[kMaxLayers][kMaxDepth];
};

// Packs every MFMA weight matrix of the model (forward W and adjoint W^T)
// from the flat float64 weight vector `base`; records byte offsets.
void pack_bf16_frags(const afm_model* m, const double* base, std::vector<char>& out, DevWeights* Wd) {
  const ModelDims& d = m->dims;
  FragOffsets fo{};
  out.clear();
  char nm[32];
  for (int k = 1; k < d.ntb; ++k) {
    snprintf(nm, sizeof nm, "twobody.%d", k);
    const afm_param_block* b = blk(m, nm);
    pack_matrix(base + b->offset, (int)b->rows, (int)b->cols, false, out, &fo.tbf[k]);
    pack_matrix(base + b->offset, (int)b->cols, (int)b->rows, true, out, &fo.tbb[k]);
  }
  for (int L = 1; L <= d.NL; ++L) {
    snprintf(nm, sizeof nm, "layer%d.env", L);
    const afm_param_block* b = blk(m, nm);
    std::vector<double> perm((size_t)b->rows * b->cols);
    for (int l = 0; l <= d.lmax; ++l)
      for (int n = 0; n < d.c; ++n)
        memcpy(&perm[((size_t)l * d.c + n) * d.w], base + b->offset + ((size_t)n * (d.lmax + 1) + l) * d.w,
               sizeof(double) * d.w);
    pack_matrix(perm.data(), (int)b->rows, d.w, false, out, &fo.envf[L - 1]);
    pack_matrix(perm.data(), d.w, (int)b->rows, true, out, &fo.envb[L - 1]);
    for (int k = 0; k < d.depth; ++k) {
      snprintf(nm, sizeof nm, "layer%d.latent.%d", L, k);
      b = blk(m, nm);
      pack_matrix(base + b->offset, (int)b->rows, (int)b->cols, false, out, &fo.latf[L - 1][k]);
      pack_matrix(base + b->offset, (int)b->cols, (int)b->rows, true, out, &fo.latb[L - 1][k]);
    }
  }
  static_assert(sizeof(FragOffsets) <= sizeof(Wd->frag_off), "offset table too small");
  memcpy(Wd->frag_off, &fo, sizeof fo);
}

// ---------------------------------------------------------------------------
// kernel arguments

struct ChainArgs {
  RowRange rr;
  const float* geo;
  const int32_t* eidx;
  const int32_t* col;
  const int32_t* species;
  const int64_t* seg;
  int64_t B;
  const double* ges;
  const double* sp_scale;
  double escale;
  int S, nb;
  float r_cut;
  const float* w0;        // first two-body layer, float32 [T0][2S + nb]
  const float* w_eff;     // [W]
  const uint4* tbf[kMaxTwobody];
  const uint4* tbb[kMaxTwobody];
  const uint4* envf;      // environment embedding (forward) used after this MLP
  const uint4* envb;      // transposed environment embedding (adjoint) used before it
  const uint4* latf[kMaxDepth];
  const uint4* latb[kMaxDepth];
  const float* xprev;     // x^{L-1}
  float* xnew;            // x^L (or x^0)
  const uint16_t* s16;   // s^L (bf16 bits)
  uint16_t* omega;        // omega^{L+1} (or omega^1), bf16 bits
  float* eps;             // edge energies (global edge index)
  uint2* pre[kMaxDepth];  // bf16 pre-activations per MLP layer
  float* gx;              // dE/dx (in: of x^L / x^0; out: of x^{L-1})
  uint16_t* gs;           // dE/ds^L (bf16)
  const uint16_t* gomega; // dE/domega^{L+1} (or of omega^1), bf16 bits
  float* gy;              // [t][16], dE/du at [9]
  float* grho;            // [t][16]
};

// ---------------------------------------------------------------------------
// dispatch over the built shapes: (w, c, l_max, depth, two-body widths, n0e)

#define AFM_SHAPES(X)                       \
  X(32, 8, 1, 2, 16, 32, 0, 2)              \
  X(64, 16, 2, 3, 16, 32, 64, 3)            \
  X(128, 32, 2, 3, 32, 64, 128, 3)          \
  X(256, 64, 2, 3, 64, 128, 256, 3)         \
  X(64, 16, 3, 3, 16, 32, 64, 4)            \
  X(256, 64, 3, 3, 64, 128, 256, 4)
// the 512-wide model (Table 1's largest: c = 128, two-body [128, 256, 512]);
// its LDS tiles fit only the 64-edge shape
#define AFM_SHAPES_WIDE(X)                  \
  X(512, 128, 2, 3, 128, 256, 512, 3)

static bool shape_is(const ModelDims& d, int w, int c, int lmax, int depth, int t0, int t1, int t2, int n0e) {
  if (d.w != w || d.c != c || d.lmax != lmax || d.depth != depth) return false;
  if (t2 ? (d.ntb != 3 || d.tb[0] != t0 || d.tb[1] != t1 || d.tb[2] != t2)
         : (d.ntb != 2 || d.tb[0] != t0 || d.tb[1] != t1))
    return false;
  const Plan P = make_plan(d.lmax, d.NL);
  for (int L = 0; L < d.NL; ++L)
    if (P.layer[L].n0e != n0e) return false;
  return d.nb <= 16;
}

int mfma_check_shape(const afm_model* m) {
#define X(w, c, l, dp, a0, a1, a2, n0)                                            \
  if (shape_is(m->dims, w, c, l, dp, a0, a1, a2, n0)) {                          \
    if (m->edge_tile == 64 || w <= 256) return AFM_OK;                           \
    set_error("latent widths above 256 are built for 64-edge tiles only");       \
    return AFM_E_UNSUPPORTED;                                                    \
  }
  AFM_SHAPES(X)
  AFM_SHAPES_WIDE(X)
#undef X
  set_error("BF16 MFMA kernels are built for (w, c, l_max, depth, two-body) = (32,8,1,2,[16,32]), "
            "(64,16,2,3,[16,32,64]), (128,32,2,3,[32,64,128]), (256,64,2,3,[64,128,256]), "
            "(64,16,3,3,[16,32,64]), (256,64,3,3,[64,128,256]), "
            "(512,128,2,3,[128,256,512]; 64-edge tiles only)");
  return AFM_E_UNSUPPORTED;
}

static ChainArgs base_args(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                           const int32_t* species) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  const char* fb = static_cast<const char*>(m->W.frag);
  ChainArgs a{};
  a.rr = rr;
  a.geo = ws_ptr<float>(ws, L.geo);
  a.eidx = ws_ptr<int32_t>(ws, L.eidx);
  a.species = species;
  a.sp_scale = m->W.sp_scale;
  a.escale = d.escale;
  a.S = d.S;
  a.nb = d.nb;
  a.r_cut = (float)d.r_cut;
  a.w0 = m->W.tb[0];
  a.w_eff = m->W.w_eff;
  for (int k = 1; k < d.ntb; ++k) {
    a.tbf[k] = reinterpret_cast<const uint4*>(fb + fo->tbf[k]);
    a.tbb[k] = reinterpret_cast<const uint4*>(fb + fo->tbb[k]);
  }
  a.gy = ws_ptr<float>(ws, L.gy);
  a.grho = ws_ptr<float>(ws, L.grho);
  a.gx = ws_ptr<float>(ws, L.gx);
  a.gomega = ws_ptr<uint16_t>(ws, L.gomega);
  return a;
}

static const uint4* frag_ptr(const afm_model* m, int64_t off) {
  return reinterpret_cast<const uint4*>(static_cast<const char*>(m->W.frag) + off);
}

// The edge-tile shapes of the chains, chosen per model (afm_set_edge_tile,
// or measured by afm_tune_edge_tile):
//   t64:   64 edges,  8 wavefronts of 4 column blocks, 4 wavefronts per SIMD
//          (two workgroups per CU);
//   t128:  128 edges, 16 wavefronts of 4 column blocks, 4 per SIMD (one
//          workgroup per CU);
//   t128w: 128 edges, 8 wavefronts of 8 column blocks, 2 per SIMD (one
//          workgroup per CU): a weight fragment feeds twice the MFMAs, so
//          the L2 weight stream per edge halves and each k-block's MFMAs
//          cover more of its loads' latency, with half the wavefronts.
namespace t64 {
constexpr int NCB = 4, NCBW = 4, WPE = 4;
#define AFM_TILE_WIDE 1
#define AFM_TILE_FUSED 1
#include "mfma_chain_tile.h"
#undef AFM_TILE_FUSED
#undef AFM_TILE_WIDE
}  // namespace t64
namespace t128 {
constexpr int NCB = 8, NCBW = 4, WPE = 4;
#include "mfma_chain_tile.h"
}  // namespace t128
namespace t128w {
constexpr int NCB = 8, NCBW = 8, WPE = 2;
#include "mfma_chain_tile.h"
}  // namespace t128w

// dispatch a launcher on the model's tile shape
#define AFM_TILE_DISPATCH(m, call) \
  ((m)->edge_tile == 128 ? ((m)->tile_waves == 8 ? t128w::call : t128::call) : t64::call)

static int checked(const afm_model* m, int rc) { return rc == AFM_E_UNSUPPORTED ? mfma_check_shape(m) : rc; }

int mfma_twobody_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, const int32_t* col, hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.col = col;
  a.envf = frag_ptr(m, fo->envf[0]);
  a.xnew = ws_ptr<float>(ws, L.x[0]);
  a.omega = ws_ptr<uint16_t>(ws, L.omega[0]);
  for (int k = 0; k < d.ntb; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.tb_pre[k]);
  return checked(m, AFM_TILE_DISPATCH(m, launch_tb_fwd(d, a, L, st)));
}

int mfma_twobody_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                     const int32_t* species, hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.envb = frag_ptr(m, fo->envb[0]);
  for (int k = 0; k < d.ntb; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.tb_pre[k]);
  const bool fast = m->fast_adjoint;
  return checked(m, AFM_TILE_DISPATCH(m, launch_tb_bwd(d, fast, a, L, st)));
}

int mfma_latent_fwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, nullptr);
  for (int k = 0; k < d.depth; ++k) a.latf[k] = frag_ptr(m, fo->latf[layer - 1][k]);
  if (layer < d.NL) a.envf = frag_ptr(m, fo->envf[layer]);
  a.xprev = ws_ptr<float>(ws, L.x[layer - 1]);
  a.xnew = layer < d.NL ? ws_ptr<float>(ws, L.x[layer]) : nullptr;
  a.s16 = ws_ptr<uint16_t>(ws, L.s[layer - 1]);
  a.omega = layer < d.NL ? ws_ptr<uint16_t>(ws, L.omega[layer]) : nullptr;
  a.eps = ws_ptr<float>(ws, L.eps);
  for (int k = 0; k < d.depth; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.lat_pre[layer - 1][k]);
  const bool last = layer == d.NL;
  return checked(m, AFM_TILE_DISPATCH(m, launch_lat_fwd(d, last, a, L, st)));
}

int mfma_latent_bwd(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr, int layer,
                    const int32_t* species, const int64_t* seg, int64_t B, const double* grad_e_struct,
                    hipStream_t st) {
  const ModelDims& d = m->dims;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.seg = seg;
  a.B = B;
  a.ges = grad_e_struct;
  a.gs = ws_ptr<uint16_t>(ws, L.gs[layer - 1]);
  for (int k = 0; k < d.depth; ++k) a.latb[k] = frag_ptr(m, fo->latb[layer - 1][k]);
  if (layer < d.NL) a.envb = frag_ptr(m, fo->envb[layer]);
  for (int k = 0; k < d.depth; ++k) a.pre[k] = ws_ptr<uint2>(ws, L.lat_pre[layer - 1][k]);
  const bool last = layer == d.NL, fast = m->fast_adjoint;
  return checked(m, AFM_TILE_DISPATCH(m, launch_lat_bwd(d, last, fast, a, L, st)));
}

// The last latent layer's forward and adjoint fused (k_lat_fb): built for
// the 64-edge tile and latent widths up to 256.
bool mfma_fused_last_available(const afm_model* m) {
  if (m->prec != AFM_BF16_MFMA || m->edge_tile != 64 || m->dims.w > 256) return false;
#define X(w, c, l, dp, a0, a1, a2, n0) \
  if (shape_is(m->dims, w, c, l, dp, a0, a1, a2, n0)) return true;
  AFM_SHAPES(X)
#undef X
  return false;
}

int mfma_latent_fb(const afm_model* m, const afm_workspace* ws, const WsLayout& L, RowRange rr,
                   const int32_t* species, const int64_t* seg, int64_t B, const double* grad_e_struct, hipStream_t st) {
  const ModelDims& d = m->dims;
  const int layer = d.NL;
  const FragOffsets* fo = reinterpret_cast<const FragOffsets*>(m->W.frag_off);
  ChainArgs a = base_args(m, ws, L, rr, species);
  a.seg = seg;
  a.B = B;
  a.ges = grad_e_struct;
  for (int k = 0; k < d.depth; ++k) {
    a.latf[k] = frag_ptr(m, fo->latf[layer - 1][k]);
    a.latb[k] = frag_ptr(m, fo->latb[layer - 1][k]);
  }
  a.xprev = ws_ptr<float>(ws, L.x[layer - 1]);
  a.s16 = ws_ptr<uint16_t>(ws, L.s[layer - 1]);
  a.eps = ws_ptr<float>(ws, L.eps);
  a.gs = ws_ptr<uint16_t>(ws, L.gs[layer - 1]);
  return checked(m, t64::launch_lat_fb(d, m->fast_adjoint, a, L, st));
}

}  // namespace afm
