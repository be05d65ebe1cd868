// Layout of the per-chunk edge buffers shared by the edge and atom kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace afm {

// geo[t][16]: delta (3, float32 from the float64 difference), |delta|,
// envelope u, the 9 spherical-harmonic components (l <= 2), 2 unused.
constexpr int GEO_D = 3, GEO_U = 4, GEO_Y = 5, GEO_STRIDE = 16;
// l_max = 3 only: geo3[t][8] holds Y^3 (7 values), gy3[t][8] its adjoint
constexpr int GEO3_STRIDE = 8;

// Row (central atom) and edge range of one chunk, read on the device.
struct RowRange {
  const int64_t* chunk_rows;
  const int64_t* row_ptr;
  int chunk;
  __device__ __forceinline__ void get(int64_t& e0, int64_t& e1) const {
    e0 = row_ptr[chunk_rows[chunk]];
    e1 = row_ptr[chunk_rows[chunk + 1]];
  }
};

// Operands of the environment-sum / tensor-product kernels of one layer.
constexpr int kMaxTpLayers = 4;

struct TPArgs {
  RowRange rr;
  const float* geo;
  // omega, s and dE/domega are float in the FP32 path and bf16 bits in the
  // BF16 path (its MLP kernels round them to bf16 anyway)
  const void* omega;     // omega^L  [t][lmax+1][C]
  const void* omega1;    // omega^1  (features V^0 = omega^1 (x) Y when L == 1)
  void* s;               // s^L      [t][n0e][C]
  float* gamma;          // Gamma^L  [N][(lmax+1)^2][C]
  const float* alpha;    // [n_paths][C]
  // every layer's per-atom sums, mixing weights and scalar-output adjoints
  // (index l: layer l + 1).  Neither V^{L-1} nor dE/dV^L is stored: the
  // forward rebuilds V^{L-1} per edge from V^0 = omega^1 (x) Y and the
  // Gammas of the earlier layers, the adjoint rebuilds dE/dV^L from the
  // later layers' Gammas and dE/ds.
  const float* gamma_l[kMaxTpLayers];
  const float* alpha_l[kMaxTpLayers];
  const void* gs_l[kMaxTpLayers];   // dE/ds: float (FP32 path) or bf16 bits
  float inv_sqrt_nbar;
  void* gomega;          // dE/domega^L [t][lmax+1][C]
  float* gy;             // dE/dY [t][16]  (+=), dE/du at [9]
  const float* geo3;     // Y^3 [t][8] (l_max = 3, else null)
  float* gy3;            // dE/dY^3 [t][8] (+=; l_max = 3, else null)
  // first channel of this launch: a launch covers channels [c0, c0 + C)
  // of the arrays' channels (the products are channelwise)
  int c0;
};

int launch_tp(int lmax, int NL, int L, int C, bool bwd, bool bf16, const TPArgs& a, int64_t n_atoms_max,
              hipStream_t st);

// Operands of the dense-mixing tensor-product kernels of layer L (per-edge
// features stored; arrays of C = channels).
struct DenseArgs {
  RowRange rr;
  const float* geo;
  const void* omega;     // omega^L  [t][lmax+1][C]  (float or bf16 bits, as in TPArgs)
  const void* omega1;    // omega^1
  void* s;               // s^L      [t][n0e][C]     (float or bf16 bits)
  float* gamma;          // Gamma^L  [N][(lmax+1)^2][C]
  const float* vin;      // V^{L-1}  [t][n_in_comps][C]  (L >= 2)
  float* tbuf;           // forward: T^L written; adjoint: dE/dT^L read  [t][T comps][C]
  float* dvbuf;          // adjoint: dE/dV^{L-1} written  [t][n_in_comps][C]
  const void* gs;        // dE/ds^L  [t][n0e][C]     (float or bf16 bits)
  void* gomega;          // dE/domega^L [t][lmax+1][C] (float or bf16 bits)
  float* gy;             // dE/dY [t][16]  (+=)
  float inv_sqrt_nbar;
};

int launch_dense_tp(int lmax, int NL, int L, int C, bool bwd, bool bf16, const DenseArgs& a,
                    int64_t n_atoms_max, hipStream_t st);
}  // namespace afm
struct afm_model;
namespace afm {
// the mixing GEMMs of layer L < N_L over a chunk of at most E edges:
// forward T (tbuf) -> V^L (feat), adjoint dE/dV^L (feat) -> dE/dT (tbuf)
int launch_dense_mix(const afm_model* m, int L, bool bwd, RowRange rr, int64_t E, float* feat, float* tbuf,
                     hipStream_t st);

}  // namespace afm
