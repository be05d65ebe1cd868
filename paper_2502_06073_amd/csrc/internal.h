// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/afm.h"
#include "plan.h"

namespace afm {

void set_error(const std::string& msg);

#define AFM_HIP_CHECK(expr)                                                   \
  do {                                                                        \
    hipError_t _e = (expr);                                                   \
    if (_e != hipSuccess) {                                                   \
      ::afm::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));    \
      return AFM_E_HIP;                                                       \
    }                                                                         \
  } while (0)

#define AFM_LAUNCH_CHECK()                                                    \
  do {                                                                        \
    hipError_t _e = hipGetLastError();                                        \
    if (_e != hipSuccess) {                                                   \
      ::afm::set_error(std::string("kernel launch: ") + hipGetErrorString(_e)); \
      return AFM_E_HIP;                                                       \
    }                                                                         \
  } while (0)

constexpr int kMaxTwobody = 4;
constexpr int kMaxDepth = 4;
constexpr int kMaxSpecies = 128;

// Device-side weights.  FP32 copies in the layouts the kernels read; the
// environment embedding rows are reordered l-major (row l*c + n holds the
// paper-order row n*(l_max+1) + l) so that omega is stored [l][c] per edge.
struct DevWeights {
  const float* tb[kMaxTwobody] = {};           // [out][in]
  const float* env[kMaxLayers] = {};           // [(lmax+1)*c][w], l-major rows
  const float* lat[kMaxLayers][kMaxDepth] = {};// [out][in]
  const float* alpha[kMaxLayers] = {};         // [n_paths][c]
  // dense mixing: per output irrep r of layer L, A_r [c][np_r c] (column
  // block j: the j-th path into r, in path order) at mix[L-1] + mix_off[L-1][r]
  const float* mix[kMaxLayers] = {};
  int64_t mix_off[kMaxLayers][kMaxIrreps] = {};
  // BF16 models: the same matrices as bf16 pairs w = hi + lo, four arrays
  // of mix_elems[L] values each: [hi | lo] of A_r, then [hi | lo] of A_r^T
  // ([np_r c][c]), every A_r at element offset mix_off[L-1][r]
  const uint16_t* mix_b16[kMaxLayers] = {};
  int64_t mix_elems[kMaxLayers] = {};
  const float* w_eff = nullptr;                // [w] = W_E1^T W_E2^T
  const float* e0 = nullptr;                   // [h][w]
  const float* e1 = nullptr;                   // [h]
  const double* sp_scale = nullptr;            // [S]
  const double* sp_shift = nullptr;            // [S]
  // BF16 MFMA fragment-packed copies (see mfma_chain.hip); null for FP32
  const void* frag = nullptr;
  int64_t frag_off[64] = {};   // byte offsets of the packed matrices in `frag`
};

struct ModelDims {
  int S, lmax, NL, w, c, nb, p, ntb, depth, h;
  int tb[kMaxTwobody];
  int n_lm;             // (lmax+1)^2 spherical-harmonic components
  bool dense;           // dense channel-mixing matrices after the products
  double r_cut, nbar, escale;
};

}  // namespace afm

struct afm_model {
  uint64_t uid = 0;            // creation id, never reused (graph cache key)
  afm_hparams hp;
  afm_precision prec;          // AFM_FP32_PLAIN or AFM_BF16_MFMA
  bool fast_adjoint = false;   // AFM_BF16_MFMA_FAST_ADJOINT was asked for
  bool fuse_last = true;       // fused last-layer forward + adjoint where built
  int edge_tile = 64;          // edges per workgroup tile of the BF16 MFMA chains (64 or 128)
  int tile_waves = 8;          // wavefronts per workgroup (64: 8; 128: 16 or 8)
  afm::ModelDims dims;
  afm::Plan plan;
  int device;
  int64_t n_params;
  std::vector<afm_param_block> blocks;
  void* dev_mem = nullptr;
  int64_t dev_bytes = 0;
  afm::DevWeights W;
};

namespace afm {

// Byte layout of a workspace, derived deterministically from the model and
// the afm_workspace fields.  Offsets are relative to ws->ptr.
struct WsLayout {
  int64_t total = 0;
  // neighbour-list scratch
  int64_t nb_struct = 0, nb_atom = 0, nb_bin_count = 0, nb_bin_start = 0,
          nb_bin_atoms = 0, nb_counts = 0, nb_scan = 0;
  int64_t n_bins_max = 0;
  // chunking
  int64_t chunk_rows = 0;      // int64 [n_chunks + 1]
  // global per-edge / per-atom buffers
  int64_t g = 0;               // float [capacity][3]
  int64_t gamma[kMaxLayers] = {};  // float [N][n_lm][c]
  int64_t eps = 0;             // float [capacity] edge energies
  int64_t atom_virial = 0;     // double [N][9]
  int64_t md_ref = 0;          // double [N][3] positions at the last rebuild
  int64_t md_ke = 0;           // double [ceil(N/256)] kinetic-energy partials
  // edge list restricted to |delta| < r_c (MD with a skin)
  int64_t c_row_ptr = 0;       // int64 [N + 1]
  int64_t c_col = 0, c_rev = 0, c_map = 0, c_idx = 0;  // int32 [capacity]
  int64_t c_shift = 0;         // int8 [capacity][3]
  int64_t c_flag = 0;          // uint8 [capacity]
  int64_t c_n_edges = 0;       // int64 [1]
  // per-chunk edge buffers (CEX edges)
  int64_t cex = 0;
  int64_t eidx = 0;            // int32 [CEX] central atom of each local edge
  int64_t geo = 0;             // float [CEX][16]
  int64_t tb_pre[kMaxTwobody] = {};          // float [CEX][tb_k]
  int64_t x[kMaxLayers + 1] = {};            // float [CEX][w]  x^0..x^{NL-1}
  int64_t omega[kMaxLayers] = {};            // float [CEX][(lmax+1)c]
  int64_t s[kMaxLayers] = {};                // float [CEX][n0e c]
  int64_t lat_pre[kMaxLayers][kMaxDepth] = {};  // float [CEX][w] (BF16 path: bf16)
  int64_t gx = 0, gt0 = 0, gt1 = 0;          // float [CEX][max(w, w+n0e c)]
  int64_t gs[kMaxLayers] = {};               // float [CEX][n0e c] dE/ds^L per layer
  int64_t gy = 0;                            // float [CEX][16] (GY[9], Gu at [9])
  int64_t gomega = 0;                        // float [CEX][(lmax+1)c]
  int64_t grho = 0;                          // float [CEX][16]
  int64_t geo3 = 0, gy3 = 0;                 // float [CEX][8] Y^3 and dE/dY^3 (l_max = 3 only)
  // dense mixing only: V^L [CEX][n_out_comps][c] (L < NL), the products T
  // (forward) or their adjoints (backward) [CEX][t comps][c], and dE/dV^{L-1}
  // [CEX][n_in_comps][c]
  int64_t dense_v[kMaxLayers] = {}, dense_t = 0, dense_dv = 0;
  // second order (stacked rows: primal [0, CEX), tangent [CEX, 2 CEX))
  int64_t so_geo2 = 0;                                   // float [CEX][16]
  int64_t so_tb_pre[kMaxTwobody] = {};                   // float [2CEX][tb_k]
  int64_t so_x[kMaxLayers + 1] = {};                     // float [2CEX][w]
  int64_t so_omega[kMaxLayers] = {};                     // float [2CEX][(lmax+1)c]
  int64_t so_s[kMaxLayers] = {};                         // float [2CEX][n0e c]
  int64_t so_v[kMaxLayers] = {};                         // float [2CEX][ncomp c]
  int64_t so_lat_pre[kMaxLayers][kMaxDepth] = {};        // float [2CEX][w]
  int64_t so_gammad[kMaxLayers] = {};                    // float [N][n_lm][c]
  int64_t so_gx = 0, so_ga = 0, so_gh = 0;               // float [2CEX][wide]
  int64_t so_gs = 0;                                     // float [2CEX][n0e c]
  int64_t so_gv0 = 0, so_gv1 = 0;                        // float [2CEX][maxcomp c]
  int64_t so_gomega = 0;                                 // float [2CEX][(lmax+1)c]
  int64_t so_eps = 0, so_coef = 0;                       // float [2CEX]
  int64_t so_partial = 0;                                // float [32][max |W|]
  int64_t so_gacc = 0;                                   // double [n_params]
  int64_t so_q = 0;                                      // double [w]
  int64_t so_galpha[kMaxLayers] = {};                    // float [N][n_paths][c]
  int64_t so_asig = 0, so_amu = 0;                       // double [N]
  int64_t so_badj = 0;                                   // float [2CEX][32] basis adjoints (position gradient)
  int64_t so_gpos = 0;                                   // float [capacity][3] dJ/d delta_e
};

WsLayout workspace_layout(const afm_model* m, const afm_workspace* ws);

template <class T>
inline T* ws_ptr(const afm_workspace* ws, int64_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws->ptr) + off);
}

int pack_weights(afm_model* m, const double* w);   // weights.cpp

// ---- kernel launchers (defined in the .hip files) ----

struct SysDev {
  int64_t N, B;
  const double* pos;
  const int32_t* species;
  const double* cell;
  const uint8_t* pbc;
  const int64_t* seg;
};

struct NlDev {
  int64_t capacity;
  int64_t* row_ptr;
  int32_t* col;
  int8_t* shift;
  int32_t* rev;
  int64_t* n_edges;
  int32_t* status;
};

int launch_build_neighbors(const SysDev& s, double r_list, const NlDev& nl,
                           const afm_workspace* ws, const WsLayout& L, int n_species,
                           hipStream_t st);
// `out` (workspace-backed, same capacity and status as `in`) = the edges of
// `in` with |delta| < r_cut, row order kept, rev remapped.
int launch_compact_to_cutoff(const SysDev& s, const NlDev& in, float r_cut, const afm_workspace* ws,
                             const WsLayout& L, NlDev* out, hipStream_t st);

// chunk boundaries (rows) from row_ptr
int launch_chunk_rows(const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                      const WsLayout& L, hipStream_t st);

// forward/backward orchestration for one chunk (forward.hip)
// fused_last: the forward runs the last latent layer together with its
// adjoint (energy + forces call), and the backward then starts at that
// layer's tensor-product adjoint
int run_forward_chunk(const afm_model* m, const SysDev& s, const NlDev& nl,
                      const afm_workspace* ws, const WsLayout& L, int chunk,
                      hipStream_t st, bool fused_last = false);
int run_backward_chunk(const afm_model* m, const SysDev& s, const NlDev& nl,
                       const afm_workspace* ws, const WsLayout& L, int chunk,
                       const double* grad_e_struct, hipStream_t st, bool fused_last = false);
bool mfma_fused_last_available(const afm_model* m);
int run_atom_energy(const afm_model* m, const SysDev& s, const NlDev& nl,
                    const afm_workspace* ws, const WsLayout& L, double* e_atom,
                    double* e_struct, hipStream_t st);
int md_step(const afm_model* m, const SysDev& s, const NlDev& n, afm_md_state* state, int32_t n_steps,
            const afm_workspace* ws, const WsLayout& L, hipStream_t st);   // md.hip
// destroys the cached MD graphs captured with the model of this id (md.hip)
void md_evict_model(uint64_t model_uid);
int64_t md_cached_graphs();
int check_chunks(const SysDev& s, const NlDev& nl, const afm_workspace* ws, const WsLayout& L,
                 hipStream_t st);                                          // neighbors.hip

int run_second_order(const afm_model* m, const SysDev& s, const NlDev& nl, const afm_workspace* ws,
                     const WsLayout& L, const double* gE, const double* gF, const double* gW,
                     float* grad_out, double* grad_pos, hipStream_t st);                    // second_order.hip
// out_i = sum_{e in row i} (g_e - g_rev(e)), g [capacity][3] (forward.hip)
int run_edge_scatter(const SysDev& s, const NlDev& nl, const float* g, double* out, hipStream_t st);

// device address of the no-allocation entry point's static scratch array on
// `device` (static_scratch.hip); resolved once per device
int static_scratch_resolve(int device, void** out);

int run_force_scatter(const afm_model* m, const SysDev& s, const NlDev& nl,
                      const afm_workspace* ws, const WsLayout& L, double* forces,
                      double* virial, hipStream_t st);

}  // namespace afm
