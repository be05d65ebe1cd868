// Host side of the library: hyperparameter checks, the flat weight layout,
// the real Clebsch-Gordan tables, model creation and workspace planning.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <atomic>
#include <complex>
#include <string>
#include <vector>

#include "cg_ct.h"
#include "edge_layout.h"
#include "internal.h"

namespace afm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// ----------------------------------------------------------------------------
// hyperparameters

static int dims_of(const afm_hparams* hp, ModelDims* d) {
  if (!hp) { set_error("null hparams"); return AFM_E_INVALID; }
  if (hp->n_species < 1 || hp->n_species > kMaxSpecies) { set_error("n_species out of range"); return AFM_E_INVALID; }
  if (hp->l_max < 0 || hp->l_max > kMaxLmax) { set_error("l_max must be 0..3"); return AFM_E_UNSUPPORTED; }
  if (hp->n_layers < 1 || hp->n_layers > 3) { set_error("n_layers must be 1..3"); return AFM_E_UNSUPPORTED; }
  if (hp->n_twobody < 1 || hp->n_twobody > kMaxTwobody) { set_error("n_twobody must be 1..4"); return AFM_E_INVALID; }
  if (hp->latent_depth < 1 || hp->latent_depth > kMaxDepth) { set_error("latent_depth must be 1..4"); return AFM_E_INVALID; }
  if (hp->latent < 8 || hp->latent % 8) { set_error("latent width must be a positive multiple of 8"); return AFM_E_INVALID; }
  if (hp->twobody[hp->n_twobody - 1] != hp->latent) { set_error("last two-body width must equal latent"); return AFM_E_INVALID; }
  for (int k = 0; k < hp->n_twobody; ++k)
    if (hp->twobody[k] < 1) { set_error("bad two-body width"); return AFM_E_INVALID; }
  if (hp->channels != 8 && hp->channels != 16 && hp->channels != 32 && hp->channels != 64 && hp->channels != 128) {
    set_error("channels must be 8, 16, 32, 64 or 128"); return AFM_E_UNSUPPORTED;
  }
  if (hp->l_max == 3 && (hp->n_layers > 2 || (hp->channels != 16 && hp->channels != 64))) {
    set_error("l_max = 3 is built for 1 or 2 layers and 16 or 64 channels"); return AFM_E_UNSUPPORTED;
  }
  if (hp->mixing != 0 && hp->mixing != 1) { set_error("mixing must be 0 (per path) or 1 (dense)"); return AFM_E_INVALID; }
  if (hp->mixing == 1 && (hp->l_max > 2 || hp->channels > 64)) {
    set_error("dense mixing is built for l_max <= 2 and channels <= 64"); return AFM_E_UNSUPPORTED;
  }
  if (hp->n_bessel < 1 || hp->n_bessel > 16) { set_error("n_bessel must be 1..16"); return AFM_E_INVALID; }
  if (hp->poly_p < 2) { set_error("poly_p must be >= 2"); return AFM_E_INVALID; }
  if (hp->edge_hidden < 1) { set_error("edge_hidden must be >= 1"); return AFM_E_INVALID; }
  if (!(hp->r_cut > 0) || !(hp->avg_num_neighbors > 0) || !isfinite(hp->energy_scale)) {
    set_error("r_cut, avg_num_neighbors must be positive, energy_scale finite"); return AFM_E_INVALID;
  }
  d->S = hp->n_species; d->lmax = hp->l_max; d->NL = hp->n_layers; d->w = hp->latent;
  d->c = hp->channels; d->nb = hp->n_bessel; d->p = hp->poly_p; d->ntb = hp->n_twobody;
  d->depth = hp->latent_depth; d->h = hp->edge_hidden;
  for (int k = 0; k < kMaxTwobody; ++k) d->tb[k] = k < hp->n_twobody ? hp->twobody[k] : 0;
  d->n_lm = (hp->l_max + 1) * (hp->l_max + 1);
  d->r_cut = hp->r_cut; d->nbar = hp->avg_num_neighbors; d->escale = hp->energy_scale;
  d->dense = hp->mixing == 1;
  return AFM_OK;
}

static void push_block(std::vector<afm_param_block>& v, const char* name, int64_t rows,
                       int64_t cols, int64_t fan_in, int init, int64_t& off) {
  afm_param_block b{};
  strncpy(b.name, name, sizeof(b.name) - 1);
  b.offset = off; b.rows = rows; b.cols = cols; b.fan_in = fan_in; b.init = init;
  off += rows * cols;
  v.push_back(b);
}

static int build_layout(const afm_hparams* hp, std::vector<afm_param_block>& out, int64_t* total) {
  ModelDims d{};
  int rc = dims_of(hp, &d);
  if (rc) return rc;
  Plan P = make_plan(d.lmax, d.NL);
  if (!P.ok) { set_error("unsupported (l_max, n_layers)"); return AFM_E_UNSUPPORTED; }
  out.clear();
  int64_t off = 0;
  char nm[32];
  int64_t in = 2 * d.S + d.nb;
  for (int k = 0; k < d.ntb; ++k) {
    snprintf(nm, sizeof nm, "twobody.%d", k);
    push_block(out, nm, d.tb[k], in, in, 0, off);
    in = d.tb[k];
  }
  for (int L = 1; L <= d.NL; ++L) {
    const LayerPlan& lp = P.layer[L - 1];
    snprintf(nm, sizeof nm, "layer%d.env", L);
    push_block(out, nm, (int64_t)d.c * (d.lmax + 1), d.w, d.w, 0, off);
    int64_t lin = d.w + (int64_t)lp.n0e * d.c;
    for (int k = 0; k < d.depth; ++k) {
      snprintf(nm, sizeof nm, "layer%d.latent.%d", L, k);
      push_block(out, nm, d.w, k ? d.w : lin, k ? d.w : lin, 0, off);
    }
    if (L < d.NL && d.dense) {
      snprintf(nm, sizeof nm, "layer%d.mix", L);
      push_block(out, nm, (int64_t)lp.n_paths * d.c, d.c, d.c, 0, off);
    } else if (L < d.NL) {
      snprintf(nm, sizeof nm, "layer%d.alpha", L);
      push_block(out, nm, lp.n_paths, d.c, 1, 2, off);
    }
  }
  push_block(out, "edge.0", d.h, d.w, d.w, 0, off);
  push_block(out, "edge.1", 1, d.h, d.h, 0, off);
  push_block(out, "species.scale", d.S, 1, 1, 2, off);
  push_block(out, "species.shift", d.S, 1, 1, 1, off);
  *total = off;
  return AFM_OK;
}

// ----------------------------------------------------------------------------
// Real Clebsch-Gordan tensors.  Complex coefficients from Racah's closed
// formula, moved to the real basis Y_real = U Y_complex of spherical
// harmonics without the Condon-Shortley phase (l = 1 ordered (y, z, x)),
// normalised to sum C^2 = 2 l3 + 1, sign fixed by the first nonzero entry.

static double fact(int n) {
  double r = 1;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

static double cg_complex(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || abs(m1) > j1 || abs(m2) > j2 || abs(M) > J) return 0.0;
  if (J < abs(j1 - j2) || J > j1 + j2) return 0.0;
  double pre = sqrt((2 * J + 1) * fact(J + j1 - j2) * fact(J - j1 + j2) * fact(j1 + j2 - J) /
                    fact(j1 + j2 + J + 1));
  pre *= sqrt(fact(J + M) * fact(J - M) * fact(j1 - m1) * fact(j1 + m1) * fact(j2 - m2) *
              fact(j2 + m2));
  double s = 0;
  for (int k = 0; k <= j1 + j2 + J; ++k) {
    int a = j1 + j2 - J - k, b = j1 - m1 - k, c = j2 + m2 - k, d = J - j2 + m1 + k,
        e = J - j1 - m2 + k;
    if (a < 0 || b < 0 || c < 0 || d < 0 || e < 0) continue;
    s += ((k & 1) ? -1.0 : 1.0) / (fact(k) * fact(a) * fact(b) * fact(c) * fact(d) * fact(e));
  }
  return pre * s;
}

typedef std::complex<double> cd;

static void real_basis(int l, std::vector<cd>& U) {
  int d = 2 * l + 1;
  U.assign(d * d, cd(0, 0));
  const double r2 = 1.0 / sqrt(2.0);
  for (int m = -l; m <= l; ++m) {
    int r = m + l;
    if (m == 0) {
      U[r * d + l] = 1.0;
    } else if (m > 0) {
      U[r * d + l + m] = ((m & 1) ? -1.0 : 1.0) * r2;
      U[r * d + l - m] = r2;
    } else {
      int am = -m;
      U[r * d + l + am] = cd(0, -((am & 1) ? -1.0 : 1.0) * r2);
      U[r * d + l - am] = cd(0, r2);
    }
  }
}

int real_cg(int l1, int l2, int l3, double* out) {
  if (l1 < 0 || l2 < 0 || l3 < 0 || l3 < abs(l1 - l2) || l3 > l1 + l2 || l1 > 6 || l2 > 6)
    return AFM_E_INVALID;
  int d1 = 2 * l1 + 1, d2 = 2 * l2 + 1, d3 = 2 * l3 + 1;
  std::vector<cd> U1, U2, U3;
  real_basis(l1, U1); real_basis(l2, U2); real_basis(l3, U3);
  std::vector<cd> Cr(d1 * d2 * d3, cd(0, 0));
  for (int i = 0; i < d1; ++i)
    for (int j = 0; j < d2; ++j)
      for (int k = 0; k < d3; ++k) {
        cd acc(0, 0);
        for (int a = 0; a < d1; ++a) {
          if (U1[i * d1 + a] == cd(0, 0)) continue;
          for (int b = 0; b < d2; ++b) {
            if (U2[j * d2 + b] == cd(0, 0)) continue;
            int c = (a - l1) + (b - l2) + l3;
            if (c < 0 || c >= d3) continue;
            double cc = cg_complex(l1, a - l1, l2, b - l2, l3, c - l3);
            if (cc == 0) continue;
            acc += std::conj(U1[i * d1 + a]) * std::conj(U2[j * d2 + b]) * U3[k * d3 + c] * cc;
          }
        }
        Cr[(i * d2 + j) * d3 + k] = acc;
      }
  double mr = 0, mi = 0;
  for (auto& z : Cr) { mr = fmax(mr, fabs(z.real())); mi = fmax(mi, fabs(z.imag())); }
  bool use_imag = mi > mr;
  double ss = 0;
  for (int q = 0; q < d1 * d2 * d3; ++q) {
    double v = use_imag ? Cr[q].imag() : Cr[q].real();
    if (fabs(v) < 1e-14) v = 0.0;
    out[q] = v;
    ss += v * v;
  }
  double sc = sqrt(d3 / ss);
  double first = 0;
  for (int q = 0; q < d1 * d2 * d3; ++q) {
    out[q] *= sc;
    if (first == 0 && fabs(out[q]) > 1e-9) first = out[q];
  }
  if (first < 0)
    for (int q = 0; q < d1 * d2 * d3; ++q) out[q] = -out[q] + 0.0;
  return AFM_OK;
}

// the kernels' compile-time tables must equal the runtime derivation
static bool cg_tables_agree() {
  double buf[343];
  for (int a = 0; a <= kMaxLmax; ++a)
    for (int b = 0; b <= kMaxLmax; ++b)
      for (int c = abs(a - b); c <= a + b && c <= kMaxLmax; ++c) {
        real_cg(a, b, c, buf);
        const ct::Tensor T = ct::real_cg(a, b, c);
        for (int q = 0; q < (2 * a + 1) * (2 * b + 1) * (2 * c + 1); ++q)
          if (fabs(T.v[q] - buf[q]) > 1e-12) return false;
      }
  return true;
}

// ----------------------------------------------------------------------------
// workspace layout

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

WsLayout workspace_layout(const afm_model* m, const afm_workspace* ws) {
  WsLayout L{};
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off += align256(bytes > 0 ? bytes : 1);
    return o;
  };
  const int64_t N = ws->n_atoms, B = ws->n_struct, cap = ws->edge_capacity;
  L.n_bins_max = N + 27 * B + 1;
  L.nb_struct = take(B * 128);
  L.nb_atom = take(N * 16);
  L.nb_bin_count = take((L.n_bins_max + 1) * 4);
  L.nb_bin_start = take((L.n_bins_max + 1) * 4);
  L.nb_bin_atoms = take(N * 4);
  L.nb_counts = take((N + 1) * 8);
  L.nb_scan = take(((N + 27 * B + 2) / 1024 + 4) * 8 + 4096);
  L.chunk_rows = take((ws->n_chunks + 1) * 8);
  if (!m) { L.total = off; return L; }   // neighbour-list part only
  const ModelDims& d = m->dims;
  const Plan& P = m->plan;
  L.g = take(cap * 12);
  for (int l = 0; l < d.NL; ++l) L.gamma[l] = take(N * d.n_lm * d.c * 4);
  L.eps = take(cap * 4);
  L.atom_virial = take(N * 72);
  L.md_ref = take(N * 24);
  L.md_ke = take(((N + 255) / 256 + 1) * 8);
  L.c_row_ptr = take((N + 1) * 8);
  L.c_col = take(cap * 4);
  L.c_rev = take(cap * 4);
  L.c_map = take(cap * 4);
  L.c_idx = take(cap * 4);
  L.c_shift = take(cap * 3);
  L.c_flag = take(cap);
  L.c_n_edges = take(8);
  // per-chunk edge buffers hold whole 256-edge tiles
  const int64_t E = ((ws->n_chunks > 1 ? ws->chunk_edges + ws->max_row : cap) + 255) / 256 * 256;
  L.cex = E;
  int maxcomp = 1, maxn0 = 1;
  for (int l = 0; l < d.NL; ++l) {
    maxcomp = maxcomp > P.layer[l].n_in_comps ? maxcomp : P.layer[l].n_in_comps;
    maxcomp = maxcomp > P.layer[l].n_out_comps ? maxcomp : P.layer[l].n_out_comps;
    maxn0 = maxn0 > P.layer[l].n0e ? maxn0 : P.layer[l].n0e;
  }
  const int64_t wide = d.w + (int64_t)maxn0 * d.c;
  const int64_t gwide = wide > d.tb[0] ? wide : d.tb[0];
  const int pre_bytes = (m->prec == AFM_BF16_MFMA) ? 2 : 4;
  L.eidx = take(E * 4);
  L.geo = take(E * 64);
  for (int k = 0; k < d.ntb; ++k) L.tb_pre[k] = take(E * d.tb[k] * pre_bytes);
  for (int l = 0; l < d.NL; ++l) L.x[l] = take(E * d.w * 4);
  for (int l = 0; l < d.NL; ++l) L.omega[l] = take(E * (d.lmax + 1) * d.c * 4);
  for (int l = 0; l < d.NL; ++l) L.s[l] = take(E * (int64_t)P.layer[l].n0e * d.c * 4);
  for (int l = 0; l < d.NL; ++l)
    for (int k = 0; k < d.depth; ++k) L.lat_pre[l][k] = take(E * d.w * pre_bytes);
  L.gx = take(E * gwide * 4);
  L.gt0 = take(E * gwide * 4);
  L.gt1 = take(E * gwide * 4);
  for (int l = 0; l < d.NL; ++l) L.gs[l] = take(E * (int64_t)P.layer[l].n0e * d.c * 4);
  L.gy = take(E * 64);
  L.gomega = take(E * (d.lmax + 1) * d.c * 4);
  L.grho = take(E * 64);
  if (d.lmax == 3) {
    L.geo3 = take(E * GEO3_STRIDE * 4);
    L.gy3 = take(E * GEO3_STRIDE * 4);
  }
  if (d.dense && d.NL > 1) {
    int nt = 1, nin = 1;
    for (int l = 0; l < d.NL; ++l) {
      nt = nt > dense_t_comps(P.layer[l]) ? nt : dense_t_comps(P.layer[l]);
      nin = nin > P.layer[l].n_in_comps ? nin : P.layer[l].n_in_comps;
    }
    for (int l = 0; l + 1 < d.NL; ++l) L.dense_v[l] = take(E * (int64_t)P.layer[l].n_out_comps * d.c * 4);
    L.dense_t = take(E * (int64_t)nt * d.c * 4);
    L.dense_dv = take(E * (int64_t)nin * d.c * 4);
  }
  if (ws->with_second_order) {
    const int64_t E2 = 2 * E;
    const int envw = (d.lmax + 1) * d.c;
    L.so_geo2 = take(E * 64);
    for (int k = 0; k < d.ntb; ++k) L.so_tb_pre[k] = take(E2 * d.tb[k] * 4);
    for (int l = 0; l <= d.NL; ++l) L.so_x[l] = take(E2 * d.w * 4);
    for (int l = 0; l < d.NL; ++l) L.so_omega[l] = take(E2 * envw * 4);
    for (int l = 0; l < d.NL; ++l) L.so_s[l] = take(E2 * (int64_t)P.layer[l].n0e * d.c * 4);
    for (int l = 0; l + 1 < d.NL; ++l) L.so_v[l] = take(E2 * (int64_t)P.layer[l].n_out_comps * d.c * 4);
    for (int l = 0; l < d.NL; ++l)
      for (int k = 0; k < d.depth; ++k) L.so_lat_pre[l][k] = take(E2 * d.w * 4);
    for (int l = 0; l < d.NL; ++l) L.so_gammad[l] = take(N * d.n_lm * d.c * 4);
    L.so_gx = take(E2 * gwide * 4);
    L.so_ga = take(E2 * gwide * 4);
    L.so_gh = take(E2 * gwide * 4);
    L.so_gs = take(E2 * (int64_t)maxn0 * d.c * 4);
    L.so_gv0 = take(E2 * (int64_t)maxcomp * d.c * 4);
    L.so_gv1 = take(E2 * (int64_t)maxcomp * d.c * 4);
    L.so_gomega = take(E2 * envw * 4);
    L.so_eps = take(E2 * 4);
    L.so_coef = take(E2 * 4);
    int64_t maxw = (int64_t)d.w * (d.w + maxn0 * d.c);
    maxw = maxw > (int64_t)envw * d.w ? maxw : (int64_t)envw * d.w;
    for (int k = 0; k < d.ntb; ++k) {
      const int64_t in = k ? d.tb[k - 1] : 2 * d.S + d.nb;
      maxw = maxw > in * d.tb[k] ? maxw : in * d.tb[k];
    }
    L.so_partial = take(256 * maxw * 4);   // up to 256 row slices of one weight gradient
    L.so_gacc = take(m->n_params * 8);
    L.so_q = take((int64_t)d.w * 8);
    for (int l = 0; l + 1 < d.NL; ++l) L.so_galpha[l] = take(N * (int64_t)P.layer[l].n_paths * d.c * 4);
    L.so_asig = take(N * 8);
    L.so_amu = take(N * 8);
    L.so_badj = take(E2 * 32 * 4);
    L.so_gpos = take(cap * 12);
  }
  L.total = off;
  return L;
}

}  // namespace afm

using namespace afm;

// ============================================================================
// C ABI

extern "C" {

const char* afm_strerror(int code) {
  switch (code) {
    case AFM_OK: return "ok";
    case AFM_E_INVALID: return "invalid argument";
    case AFM_E_CAPACITY: return "buffer capacity exceeded";
    case AFM_E_NONFINITE: return "non-finite input";
    case AFM_E_UNSUPPORTED: return "unsupported precision or shape";
    case AFM_E_HIP: return "HIP runtime error";
    case AFM_E_WEIGHTS: return "weight vector does not match the layout";
    default: return "unknown error";
  }
}

const char* afm_last_error(void) { return g_last_error.c_str(); }
const char* afm_version(void) { return "afm-mi355x 0.1 (gfx950)"; }

int afm_param_layout_size(const afm_hparams* hp, int64_t* n_blocks, int64_t* n_params) {
  if (!n_blocks || !n_params) { set_error("null output"); return AFM_E_INVALID; }
  std::vector<afm_param_block> v;
  int64_t tot = 0;
  int rc = build_layout(hp, v, &tot);
  if (rc) return rc;
  *n_blocks = (int64_t)v.size();
  *n_params = tot;
  return AFM_OK;
}

int afm_param_layout_block(const afm_hparams* hp, int64_t k, afm_param_block* out) {
  if (!out) { set_error("null output"); return AFM_E_INVALID; }
  std::vector<afm_param_block> v;
  int64_t tot = 0;
  int rc = build_layout(hp, v, &tot);
  if (rc) return rc;
  if (k < 0 || k >= (int64_t)v.size()) { set_error("block index out of range"); return AFM_E_INVALID; }
  *out = v[k];
  return AFM_OK;
}

int afm_cg_real(int32_t l1, int32_t l2, int32_t l3, double* out) {
  if (!out) { set_error("null output"); return AFM_E_INVALID; }
  int rc = real_cg(l1, l2, l3, out);
  if (rc) set_error("triangle rule violated or l > 6");
  return rc;
}

int afm_model_create(const afm_hparams* hp, const double* weights, int64_t n_weights,
                     afm_precision precision, afm_model** out) {
  if (!out || !weights) { set_error("null argument"); return AFM_E_INVALID; }
  *out = nullptr;
  if (precision != AFM_FP32_PLAIN && precision != AFM_BF16_MFMA && precision != AFM_BF16_MFMA_FAST_ADJOINT) {
    set_error("precision not built (the FP64 reference is the CPU oracle)");
    return AFM_E_UNSUPPORTED;
  }
  static std::atomic<uint64_t> next_uid{1};
  afm_model* m = new afm_model();
  m->uid = next_uid.fetch_add(1);
  int rc = dims_of(hp, &m->dims);
  if (!rc) rc = build_layout(hp, m->blocks, &m->n_params);
  if (rc) { delete m; return rc; }
  if (n_weights != m->n_params) {
    set_error("expected " + std::to_string(m->n_params) + " weights, got " + std::to_string(n_weights));
    delete m;
    return AFM_E_WEIGHTS;
  }
  for (int64_t q = 0; q < n_weights; ++q)
    if (!isfinite(weights[q])) { set_error("non-finite weight"); delete m; return AFM_E_NONFINITE; }
  m->hp = *hp;
  m->fast_adjoint = precision == AFM_BF16_MFMA_FAST_ADJOINT;
  m->prec = m->fast_adjoint ? AFM_BF16_MFMA : precision;
  m->plan = make_plan(m->dims.lmax, m->dims.NL);
  // the dense kernels read V^{L-1} with layer L's input offsets from the
  // buffer written with layer L-1's output offsets
  for (int L = 2; L <= m->dims.NL && m->dims.dense; ++L) {
    const LayerPlan &a = m->plan.layer[L - 2], &b = m->plan.layer[L - 1];
    bool same = a.n_out == b.n_in && a.n_out_comps == b.n_in_comps;
    for (int r = 0; same && r < a.n_out; ++r)
      same = a.out[r].l == b.in[r].l && a.out[r].p == b.in[r].p && a.out_off[r] == b.in_off[r];
    if (!same) { set_error("internal: layer irreps do not chain"); delete m; return AFM_E_INVALID; }
  }
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); delete m; return AFM_E_HIP; }
  // library set-up on this device: the address of the no-allocation entry
  // point's scratch array (afm_energy_forces_noalloc retries and reports a
  // failure itself)
  (void)static_scratch_resolve(m->device, nullptr);
  rc = pack_weights(m, weights);
  if (rc) { if (m->dev_mem) (void)hipFree(m->dev_mem); delete m; return rc; }
  if (!cg_tables_agree()) {
    set_error("internal: compile-time and runtime CG tables differ");
    (void)hipFree(m->dev_mem);
    delete m;
    return AFM_E_INVALID;
  }
  *out = m;
  return AFM_OK;
}

int afm_stage_costs(const afm_hparams* hp, afm_stage_cost* out, int32_t max, int32_t* n) {
  if (!hp || !n || (max > 0 && !out)) { set_error("null argument"); return AFM_E_INVALID; }
  ModelDims d{};
  int rc = dims_of(hp, &d);
  if (rc) return rc;
  const Plan P = make_plan(d.lmax, d.NL);
  const double C = d.c, W = d.w, ENV = (d.lmax + 1) * d.c, NLM = (d.lmax + 1) * (d.lmax + 1);
  double tbm = (double)d.nb * d.tb[0], tbpre = d.tb[0];
  for (int k = 1; k < d.ntb; ++k) {
    tbm += (double)d.tb[k - 1] * d.tb[k];
    tbpre += d.tb[k];
  }
  std::vector<afm_stage_cost> v;
  auto add = [&](const char* name, int idx, int kind, double fl, double be, double ba) {
    afm_stage_cost c{};
    if (idx > 0) snprintf(c.name, sizeof c.name, "%s%d", name, idx);
    else snprintf(c.name, sizeof c.name, "%s", name);
    c.kind = kind;
    c.flops_per_edge = fl;
    c.bytes_per_edge = be;
    c.bytes_per_atom = ba;
    v.push_back(c);
  };
  // col + shift + two positions in, geometry record + row index out
  add("geometry", 0, 1, 60.0, 4 + 3 + 48 + 4.0 * (GEO_Y + 9) + 4, 0);
  // species pair in; x^0, omega^1 (bf16) and the stored pre-activations out
  add("twobody_fwd", 0, 0, 2.0 * (tbm + W * ENV), 8 + 4 * W + 2 * ENV + 2 * tbpre, 0);
  // dE/domega^1 (bf16), dE/dx^0, pre-activations in; dE/drho, dE/du out
  add("twobody_bwd", 0, 0, 2.0 * (tbm + W * ENV), 2 * ENV + 4 * W + 2 * tbpre + 4 * (d.nb + 1), 0);
  for (int L = 1; L <= d.NL; ++L) {
    const LayerPlan& lp = P.layer[L - 1];
    const bool last = L == d.NL;
    double nz = 0, outc = 0;
    // one real CG tensor, (2 l + 1)^3 values for l up to l_max
    std::vector<double> buf((2 * kMaxLmax + 1) * (2 * kMaxLmax + 1) * (2 * kMaxLmax + 1));
    for (int k = 0; k < lp.n_paths; ++k) {
      const PathT& t = lp.p[k];
      real_cg(t.l1, t.l2, t.l3, buf.data());
      for (int q = 0; q < (2 * t.l1 + 1) * (2 * t.l2 + 1) * (2 * t.l3 + 1); ++q) nz += std::fabs(buf[q]) > 1e-12;
      outc += 2 * t.l3 + 1;
    }
    // V^{L-1} is rebuilt from omega^1 (x) Y and the earlier layers' per-atom
    // sums, so layers after the first read omega^1 and L - 1 more Gammas
    const double prev = L == 1 ? 0.0 : ENV;
    const double gprev = (L - 1) * NLM * C;
    const double s_out = lp.n0e * C;
    // the adjoint rebuilds dE/dV^L from dE/ds and Gamma of the later layers
    double gs_later = 0.0;
    for (int l = L; l < d.NL; ++l) gs_later += P.layer[l].n0e * C;
    const double gnext = (d.NL - L) * NLM * C;
    // environment sum (NLM C fma) + nonzero CG products (2 mul + add each);
    // the recomputation of earlier layers is not counted (algorithmic work)
    double nz0 = 0;
    for (int k = 0; k < lp.n_paths; ++k) {
      const PathT& t = lp.p[k];
      if (t.s_idx < 0) continue;
      real_cg(t.l1, t.l2, t.l3, buf.data());
      for (int q = 0; q < (2 * t.l1 + 1) * (2 * t.l2 + 1) * (2 * t.l3 + 1); ++q) nz0 += std::fabs(buf[q]) > 1e-12;
    }
    if (d.dense && d.NL > 1) {
      // stored-feature kernels: V^{L-1} (or omega^1 (x) Y) in, T^L out below
      // the last layer; the mixing GEMMs over the paths with an output
      double tmix = 0;
      for (int k = 0; k < lp.n_paths; ++k)
        if (lp.p[k].out_off >= 0) tmix += 2 * lp.p[k].l3 + 1;
      const double vin = L == 1 ? 2 * ENV : 4.0 * lp.n_in_comps * C;
      const double tout = last ? 0 : 4 * tmix * C;
      add("tp_fwd", L, 1, 2 * NLM * C + 3 * nz * C + NLM * C, 2 * ENV + vin + 4 * NLM + 2 * s_out + tout,
          4 * NLM * C);
      add("tp_bwd", L, 1, 2 * NLM * C * 2 + 6 * nz * C + 2 * NLM * C,
          2 * ENV + vin + 4 * NLM + 2 * s_out + tout + 4.0 * lp.n_in_comps * C + (L == 1 ? 4 * NLM * C : 0) +
              2 * ENV + 4 * NLM,
          4 * NLM * C);
      if (!last) {
        add("mix_fwd", L, 2, 2.0 * C * C * tmix, 4 * tmix * C + 4.0 * lp.n_out_comps * C, 0);
        add("mix_bwd", L, 2, 2.0 * C * C * tmix, 4 * tmix * C + 4.0 * lp.n_out_comps * C, 0);
      }
    }
    const double tpf = 2 * NLM * C + 3 * (last ? nz0 : nz) * C + (last ? 0 : 2 * outc * C) + NLM * C;
    // omega^L, omega^1 (bf16), Y in; s^L (bf16) out
    if (!(d.dense && d.NL > 1))
      add("tp_fwd", L, 1, tpf, 2 * ENV + 4 * NLM + 2 * prev + 2 * s_out, 4 * (NLM * C + gprev));
    // adjoint: twice the products (dV and dGamma), the mixing, the environment-sum adjoint
    const double tpb = 2 * NLM * C * 2 + 6 * nz * C + (last ? 0 : 2 * outc * C) + 2 * NLM * C;
    // omega^L, omega^1, Y, dE/ds of this and the later layers in; dE/domega^L
    // (bf16) and dE/dY out
    if (!(d.dense && d.NL > 1))
      add("tp_bwd", L, 1, tpb, 2 * ENV + 4 * NLM + 2 * prev + 4 * (s_out + gs_later) + 2 * ENV + 4 * NLM,
          4 * (NLM * C + gprev + gnext));
    const double lat = (W + lp.n0e * C) * W + (d.depth - 1) * W * W;
    // x^{L-1}, s^L (bf16), u in; x^L + omega^{L+1} (bf16) or eps out; pre-activations out
    add("latent_fwd", L, 0, 2.0 * (lat + (last ? W : W * ENV)),
        4 * W + 2 * s_out + 4 + (last ? 4 : 4 * W + 2 * ENV) + 2 * d.depth * W, 0);
    // dE/domega^{L+1} (bf16), dE/dx^L, pre-activations in; dE/dx^{L-1}, dE/ds^L (bf16), dE/du out
    add("latent_bwd", L, 0, 2.0 * (lat + (last ? 0 : W * ENV)),
        (last ? 0 : 2 * ENV) + 4 * W + 2 * d.depth * W + 4 * W + 2 * s_out + 4, 0);
    // the last layer's forward and adjoint fused: x^{L-1}, s^L (bf16), u in;
    // eps, dE/dx^{L-1}, dE/ds^L (bf16), dE/du out
    if (last) add("latent_fb", L, 0, 2.0 * (lat + W) + 2.0 * lat, 4 * W + 2 * s_out + 4 + 4 + 4 * W + 2 * s_out + 4, 0);
  }
  // rho and u adjoints in, dE/d delta out
  add("geometry_bwd", 0, 1, 40.0 + 4.0 * d.nb, 4.0 * (GEO_Y + 9) + 4 * (16 + 16) + 12, 0);
  // the double backward (afm_backward_forces_backward): its GEMMs over the
  // stacked primal and tangent rows (2 per edge) -- the forward chains, then
  // per weight matrix the input-gradient and the weight-gradient products;
  // its vector-ALU tensor-product passes are not counted
  {
    double mac = 0, io = 0;   // per stacked row
    auto gemm = [&](double k, double n, int times) { mac += times * k * n; io += times * 4.0 * (k + n); };
    gemm(2.0 * d.S + d.nb, d.tb[0], 2);                       // first two-body layer, its weight gradient
    for (int k = 1; k < d.ntb; ++k) gemm(d.tb[k - 1], d.tb[k], 3);
    gemm(W, ENV, 3);                                          // env^1
    for (int L = 1; L <= d.NL; ++L) {
      const double lin = W + P.layer[L - 1].n0e * C;
      gemm(lin, W, 3);
      for (int k = 1; k < d.depth; ++k) gemm(W, W, 3);
      if (L < d.NL) gemm(W, ENV, 3);
    }
    add("second_order", 0, 0, 2.0 * 2.0 * mac, 2.0 * io, 0);
  }
  add("energy", 0, 1, 1.0, 4, 8 + 4 + 8);
  // dE/d delta of the edge and of its reverse, col, rev, shift in; forces + virial per atom out
  add("force_scatter", 0, 1, 12.0 + 18.0, 12 + 12 + 4 + 4 + 3, 24 + 72);
  *n = (int32_t)v.size();
  for (int32_t k = 0; k < max && k < (int32_t)v.size(); ++k) out[k] = v[k];
  return AFM_OK;
}

int afm_model_set_weights(afm_model* m, const double* weights, int64_t n_weights) {
  if (!m || !weights) { set_error("null argument"); return AFM_E_INVALID; }
  if (n_weights != m->n_params) {
    set_error("expected " + std::to_string(m->n_params) + " weights, got " + std::to_string(n_weights));
    return AFM_E_WEIGHTS;
  }
  for (int64_t q = 0; q < n_weights; ++q)
    if (!isfinite(weights[q])) { set_error("non-finite weight"); return AFM_E_NONFINITE; }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && dev != m->device) e = hipSetDevice(m->device);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return AFM_E_HIP; }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return AFM_E_HIP; }
  const int rc = afm::pack_weights(m, weights);
  if (dev != m->device) (void)hipSetDevice(dev);
  return rc;
}

int afm_model_destroy(afm_model* m) {
  if (!m) return AFM_OK;
  // graphs captured with this model read its weights: never replay them again
  afm::md_evict_model(m->uid);
  if (m->dev_mem) {
    hipError_t e = hipFree(m->dev_mem);
    m->dev_mem = nullptr;
    delete m;
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); return AFM_E_HIP; }
    return AFM_OK;
  }
  delete m;
  return AFM_OK;
}

int afm_workspace_plan(const afm_model* m, int64_t n_atoms, int64_t n_struct, int64_t edge_capacity,
                       int64_t max_bytes, int32_t with_second_order, afm_workspace* ws) {
  if (!ws) { set_error("null argument"); return AFM_E_INVALID; }
  if (n_atoms < 0 || n_struct < 1 || edge_capacity < 0) { set_error("bad sizes"); return AFM_E_INVALID; }
  if (edge_capacity >= (int64_t(1) << 31)) { set_error("edge capacity must be < 2^31"); return AFM_E_INVALID; }
  if (with_second_order && !m) { set_error("a second-order plan needs a model"); return AFM_E_INVALID; }
  afm_workspace w{};
  w.n_atoms = n_atoms; w.n_struct = n_struct; w.edge_capacity = edge_capacity;
  w.max_row = 1024;
  w.precision = m ? m->prec : -1;
  w.with_second_order = with_second_order;
  w.chunk_edges = edge_capacity > 0 ? edge_capacity : 1;
  w.n_chunks = 1;
  WsLayout L = workspace_layout(m, &w);
  if (m && max_bytes > 0 && L.total > max_bytes) {
    // bytes that do not scale with the chunk
    afm_workspace w1 = w;
    w1.n_chunks = 2; w1.chunk_edges = 1024;
    WsLayout L1 = workspace_layout(m, &w1);
    w1.chunk_edges = 1024 + 65536;
    WsLayout L2 = workspace_layout(m, &w1);
    double per_edge = double(L2.total - L1.total) / 65536.0;
    double fixed = double(L1.total) - per_edge * (1024 + w1.max_row);
    int64_t ce = (int64_t)((double(max_bytes) - fixed) / per_edge) - w1.max_row - 1024;
    if (ce < 4096) { set_error("max_bytes too small for a chunk of 4096 edges"); return AFM_E_CAPACITY; }
    w.chunk_edges = ce;
    w.n_chunks = (edge_capacity + ce - 1) / ce;
    if (w.n_chunks < 1) w.n_chunks = 1;
    if (w.n_chunks == 1) w.chunk_edges = edge_capacity;
    L = workspace_layout(m, &w);
  }
  w.bytes = L.total;
  w.ptr = nullptr;
  *ws = w;
  return AFM_OK;
}

}  // extern "C"
