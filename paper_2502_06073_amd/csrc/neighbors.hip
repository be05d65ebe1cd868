// Edge-list construction (the strictly-local neighbourhoods of the Abstract;
// radial cutoff of Methodology / Model Training).
//
// Output is the canonical CSR list: rows are central atoms, each row sorted
// by (j, n0, n1, n2); rev[e] indexes (j, i, -n).  The inclusion test
//   delta = (r_j - r_i) + ((n0*a + n1*b) + n2*c),  (dx*dx + dy*dy) + dz*dz < r^2
// is evaluated with explicitly rounded float64 operations, so it is the same
// bit for bit as any other evaluation in that order without fused
// multiply-adds.  Periodic images: for atoms with whole-cell offsets
// m = floor(frac(r)), the pair (i, j) tries n = k - m_j + m_i over
// |k_a| <= ceil(r / w_a) (w_a perpendicular widths) -- every image inside
// the cutoff whatever the positions.  Large periodic cells (>= 3 bins of
// width > r per axis) use a bin grid instead of all pairs.
//
// Kernels: structure prep -> bin offsets -> atom prep/binning -> bin scan ->
// bin fill -> row count -> row scan -> row fill -> per-row rank sort (binned
// rows) -> reverse index.  Deterministic: the only atomics place atoms in
// bins, and every row is sorted afterwards.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "trace.h"
#include "device_util.h"
#include "edge_geom.h"

namespace afm {

struct StructMeta {
  double inv[9];
  int32_t R[3];
  int32_t nb[3];
  int32_t mode;      // 0 = all pairs, 1 = binned, 2 = skipped (invalid cell)
  int32_t bin_off;
  int32_t nbins;
  int32_t pad[5];
};
static_assert(sizeof(StructMeta) <= 128, "StructMeta too large");

struct AtomMeta {
  int32_t m[3];
  int32_t bin;       // global bin index (binned structures), else -1
};

__device__ __forceinline__ int find_struct(const int64_t* seg, int64_t B, int64_t i) {
  int64_t lo = 0, hi = B;            // seg[lo] <= i < seg[hi]
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (seg[mid] <= i) lo = mid; else hi = mid;
  }
  return (int)lo;
}

// delta = (r_j - r_i) + ((n0 a + n1 b) + n2 c) and its squared length,
// every operation individually rounded (no contraction).
__device__ __forceinline__ double edge_d2(const double* ri, const double* rj, const double* h,
                                          int n0, int n1, int n2, bool periodic, double* dl) {
  double d2;
  double dd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double sh = 0.0;
    if (periodic)
      sh = __dadd_rn(__dadd_rn(__dmul_rn((double)n0, h[a]), __dmul_rn((double)n1, h[3 + a])),
                     __dmul_rn((double)n2, h[6 + a]));
    dd[a] = __dadd_rn(__dsub_rn(rj[a], ri[a]), sh);
  }
  d2 = __dadd_rn(__dadd_rn(__dmul_rn(dd[0], dd[0]), __dmul_rn(dd[1], dd[1])), __dmul_rn(dd[2], dd[2]));
  if (dl) { dl[0] = dd[0]; dl[1] = dd[1]; dl[2] = dd[2]; }
  return d2;
}

__global__ void k_struct_prep(const double* __restrict__ cell, const uint8_t* __restrict__ pbc,
                              const int64_t* __restrict__ seg, int64_t B, double r,
                              StructMeta* __restrict__ meta, int32_t* status) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= B) return;
  StructMeta M{};
  const int64_t ns = seg[s + 1] - seg[s];
  M.mode = 0; M.bin_off = 0; M.nbins = 0;
  if (pbc[s]) {
    const double* h = cell + 9 * s;
    double a[3] = {h[0], h[1], h[2]}, b[3] = {h[3], h[4], h[5]}, c[3] = {h[6], h[7], h[8]};
    double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double cxa[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    double axb[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double det = a[0] * bxc[0] + a[1] * bxc[1] + a[2] * bxc[2];
    if (!(fabs(det) > 1e-12) || !isfinite(det)) {
      atomicOr(status, AFM_FLAG_NONFINITE);
      M.R[0] = M.R[1] = M.R[2] = 0;
      meta[s] = M;
      return;
    }
    // inverse of the row-vector cell: frac = r . inv, inv[a][k]
    const double id = 1.0 / det;
    for (int q = 0; q < 3; ++q) {
      M.inv[q * 3 + 0] = bxc[q] * id;
      M.inv[q * 3 + 1] = cxa[q] * id;
      M.inv[q * 3 + 2] = axb[q] * id;
    }
    const double* cr[3] = {bxc, cxa, axb};
    int nb[3];
    for (int k = 0; k < 3; ++k) {
      double len = sqrt(cr[k][0] * cr[k][0] + cr[k][1] * cr[k][1] + cr[k][2] * cr[k][2]);
      double wk = fabs(det) / len;
      double q = ceil(r / wk);
      M.R[k] = (int)fmin(q, 1000.0);
      nb[k] = (int)fmin(floor(wk / (r * (1.0 + 1e-9))), 1024.0);
    }
    // a cell this thin for the cutoff is refused (it would need more than
    // 33^3 images per pair); its atoms get no edges
    if (M.R[0] > 16 || M.R[1] > 16 || M.R[2] > 16) {
      atomicOr(status, AFM_FLAG_IMAGES);
      M.mode = 2;
      M.R[0] = M.R[1] = M.R[2] = 0;
      meta[s] = M;
      return;
    }
    bool bin_ok = nb[0] >= 3 && nb[1] >= 3 && nb[2] >= 3 && ns >= 64;
    if (bin_ok) {
      const int64_t cap = ns > 27 ? ns : 27;
      while ((int64_t)nb[0] * nb[1] * nb[2] > cap) {
        int k = 0;
        if (nb[1] > nb[k]) k = 1;
        if (nb[2] > nb[k]) k = 2;
        if (nb[k] <= 3) break;
        nb[k] -= 1;
      }
      if ((int64_t)nb[0] * nb[1] * nb[2] <= cap) {
        M.mode = 1;
        M.nb[0] = nb[0]; M.nb[1] = nb[1]; M.nb[2] = nb[2];
        M.nbins = nb[0] * nb[1] * nb[2];
      }
    }
  } else {
    M.R[0] = M.R[1] = M.R[2] = 0;
  }
  meta[s] = M;
}

__global__ void k_bin_offsets(StructMeta* meta, int64_t B) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t off = 0;
  for (int64_t s = 0; s < B; ++s) {
    meta[s].bin_off = off;
    off += meta[s].mode == 1 ? meta[s].nbins : 0;
  }
}

__global__ void k_atom_prep(const double* __restrict__ pos, const int32_t* __restrict__ species,
                            const uint8_t* __restrict__ pbc, const int64_t* __restrict__ seg,
                            int64_t N, int64_t B, int n_species, const StructMeta* __restrict__ meta,
                            AtomMeta* __restrict__ am, int32_t* __restrict__ bin_count,
                            int32_t* status) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int s = find_struct(seg, B, i);
  const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  AtomMeta a{};
  a.bin = -1;
  if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) {
    atomicOr(status, AFM_FLAG_NONFINITE);
    am[i] = a;
    return;
  }
  const int32_t z = species[i];
  if (z < 0 || z >= n_species) atomicOr(status, AFM_FLAG_SPECIES);
  if (pbc[s]) {
    const StructMeta& M = meta[s];
    double f[3];
    for (int k = 0; k < 3; ++k) f[k] = p[0] * M.inv[k] + p[1] * M.inv[3 + k] + p[2] * M.inv[6 + k];
    int bb[3];
    for (int k = 0; k < 3; ++k) {
      double fl = floor(f[k]);
      if (fabs(fl) > 1e6) { atomicOr(status, AFM_FLAG_IMAGES); fl = 0; }
      a.m[k] = (int)fl;
      if (M.mode == 1) {
        int b = (int)floor((f[k] - fl) * M.nb[k]);
        b = b < 0 ? 0 : (b >= M.nb[k] ? M.nb[k] - 1 : b);
        bb[k] = b;
      }
    }
    if (M.mode == 1) {
      a.bin = M.bin_off + (bb[0] * M.nb[1] + bb[1]) * M.nb[2] + bb[2];
      atomicAdd(&bin_count[a.bin], 1);
    }
  }
  am[i] = a;
}

__global__ void k_bin_fill(const AtomMeta* __restrict__ am, int64_t N, const int32_t* __restrict__ bin_start,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ bin_atoms) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  int b = am[i].bin;
  if (b < 0) return;
  int slot = atomicAdd(&cursor[b], 1);
  bin_atoms[bin_start[b] + slot] = (int32_t)i;
}

// One wavefront per row i: the candidates (every atom of the structure
// times every image in the window, or the atoms of the 27 surrounding bins)
// are spread over the 64 lanes.  WRITE = false counts, true fills; hits of a
// 64-candidate batch are ranked by ballot, so rows of all-pairs structures
// come out in canonical (j, n) order (candidates are enumerated in that
// order) and rows of binned structures are sorted afterwards.
template <bool WRITE>
__global__ void __launch_bounds__(256) k_rows(const double* __restrict__ pos, const double* __restrict__ cell,
                                              const uint8_t* __restrict__ pbc, const int64_t* __restrict__ seg,
                                              int64_t N, int64_t B, double r2, const StructMeta* __restrict__ meta,
                                              const AtomMeta* __restrict__ am, const int32_t* __restrict__ bin_start,
                                              const int32_t* __restrict__ bin_atoms, int64_t* __restrict__ counts,
                                              const int64_t* __restrict__ row_ptr, int64_t capacity,
                                              int32_t* __restrict__ col, int8_t* __restrict__ shift,
                                              int32_t* status, int max_row) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i > N) return;
  if (i == N) {
    if (!WRITE && lane == 0) counts[N] = 0;
    return;
  }
  if (WRITE && row_ptr[N] > capacity) return;
  const int s = find_struct(seg, B, i);
  const StructMeta& M = meta[s];
  const bool periodic = pbc[s] != 0;
  const AtomMeta ai = am[i];
  if (M.mode == 2 || (M.mode == 1 && ai.bin < 0)) {
    if (!WRITE && lane == 0) counts[i] = 0;
    return;
  }
  double h[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) h[q] = periodic ? cell[9 * s + q] : 0.0;
  const double ri[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  int64_t cnt = 0;   // uniform over the wavefront
  const int64_t base = WRITE ? row_ptr[i] : 0;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  auto batch = [&](bool hit, int64_t j, int n0, int n1, int n2) {
    const uint64_t m = __ballot(hit);
    if (WRITE && hit) {
      const int64_t e = base + cnt + __popcll(m & lt);
      col[e] = (int32_t)j;
      if (n0 < -127 || n0 > 127 || n1 < -127 || n1 > 127 || n2 < -127 || n2 > 127)
        atomicOr(status, AFM_FLAG_IMAGES);
      shift[3 * e] = (int8_t)n0;
      shift[3 * e + 1] = (int8_t)n1;
      shift[3 * e + 2] = (int8_t)n2;
    }
    cnt += __popcll(m);
  };
  if (M.mode == 0) {
    const int64_t a0 = seg[s], a1 = seg[s + 1];
    const int d0 = 2 * M.R[0] + 1, d1 = 2 * M.R[1] + 1, d2 = 2 * M.R[2] + 1;
    const int64_t nimg = (int64_t)d0 * d1 * d2;
    const int64_t T = (a1 - a0) * nimg;
    for (int64_t b0 = 0; b0 < T; b0 += 64) {
      const int64_t idx = b0 + lane;
      bool hit = false;
      int64_t j = 0;
      int n0 = 0, n1 = 0, n2 = 0;
      if (idx < T) {
        j = a0 + idx / nimg;
        const int rem = (int)(idx % nimg);
        const int k0 = rem / (d1 * d2) - M.R[0], k1 = (rem / d2) % d1 - M.R[1], k2 = rem % d2 - M.R[2];
        const AtomMeta aj = am[j];
        n0 = periodic ? k0 + ai.m[0] - aj.m[0] : 0;
        n1 = periodic ? k1 + ai.m[1] - aj.m[1] : 0;
        n2 = periodic ? k2 + ai.m[2] - aj.m[2] : 0;
        if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
          const double rj[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
          hit = edge_d2(ri, rj, h, n0, n1, n2, periodic, nullptr) < r2;
        }
      }
      batch(hit, j, n0, n1, n2);
    }
  } else {
    // lane b < 27: surrounding bin b (offsets -1..1 per axis), its atoms,
    // the wrap of the bin index, and the exclusive prefix of the counts
    int st = 0, ct = 0, w0 = 0, w1 = 0, w2 = 0;
    if (lane < 27) {
      const int lb = ai.bin - M.bin_off;
      const int b2 = lb % M.nb[2], b1 = (lb / M.nb[2]) % M.nb[1], b0 = lb / (M.nb[2] * M.nb[1]);
      int p0 = b0 + lane / 9 - 1, p1 = b1 + (lane / 3) % 3 - 1, p2 = b2 + lane % 3 - 1;
      w0 = p0 < 0 ? -1 : (p0 >= M.nb[0] ? 1 : 0);
      w1 = p1 < 0 ? -1 : (p1 >= M.nb[1] ? 1 : 0);
      w2 = p2 < 0 ? -1 : (p2 >= M.nb[2] ? 1 : 0);
      p0 -= w0 * M.nb[0]; p1 -= w1 * M.nb[1]; p2 -= w2 * M.nb[2];
      const int gb = M.bin_off + (p0 * M.nb[1] + p1) * M.nb[2] + p2;
      st = bin_start[gb];
      ct = bin_start[gb + 1] - st;
    }
    int inc = ct;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    const int excl = inc - ct;
    const int T = __shfl(inc, 26, 64);
    for (int b0 = 0; b0 < T; b0 += 64) {
      const int idx = b0 + lane;
      // bin of candidate idx: the last b with excl_b <= idx
      int lo = 0, hi = 27;
#pragma unroll
      for (int it = 0; it < 5; ++it) {
        const int mid = (lo + hi) >> 1;
        if (__shfl(excl, mid, 64) <= idx) lo = mid; else hi = mid;
      }
      const int sb = __shfl(st, lo, 64), eb = __shfl(excl, lo, 64);
      const int x0 = __shfl(w0, lo, 64), x1 = __shfl(w1, lo, 64), x2 = __shfl(w2, lo, 64);
      bool hit = false;
      int64_t j = 0;
      int n0 = 0, n1 = 0, n2 = 0;
      if (idx < T) {
        j = bin_atoms[sb + (idx - eb)];
        const AtomMeta aj = am[j];
        n0 = x0 - aj.m[0] + ai.m[0];
        n1 = x1 - aj.m[1] + ai.m[1];
        n2 = x2 - aj.m[2] + ai.m[2];
        if (!(j == i && n0 == 0 && n1 == 0 && n2 == 0)) {
          const double rj[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
          hit = edge_d2(ri, rj, h, n0, n1, n2, true, nullptr) < r2;
        }
      }
      batch(hit, j, n0, n1, n2);
    }
  }
  if (!WRITE && lane == 0) {
    counts[i] = cnt;
    if (cnt > max_row) atomicOr(status, AFM_FLAG_CAPACITY);
  }
}

__device__ __forceinline__ uint64_t edge_key(int32_t j, const int8_t* n) {
  return ((uint64_t)(uint32_t)j << 24) | ((uint64_t)(uint8_t)(n[0] + 128) << 16) |
         ((uint64_t)(uint8_t)(n[1] + 128) << 8) | (uint64_t)(uint8_t)(n[2] + 128);
}

// Rank sort of the rows of binned structures: one wavefront per row.
constexpr int kSortMax = 1024;
__global__ void __launch_bounds__(256) k_row_sort(const int64_t* __restrict__ seg, int64_t N, int64_t B,
                                                  const StructMeta* __restrict__ meta,
                                                  const int64_t* __restrict__ row_ptr, int64_t capacity,
                                                  int32_t* __restrict__ col, int8_t* __restrict__ shift) {
  __shared__ uint64_t keys[4][kSortMax];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * 4 + wave;
  bool active = i < N && row_ptr[N] <= capacity;
  int64_t e0 = 0;
  int n = 0;
  if (active) {
    const int s = find_struct(seg, B, i);
    e0 = row_ptr[i];
    n = (int)(row_ptr[i + 1] - e0);
    active = meta[s].mode == 1 && n >= 2 && n <= kSortMax;
  }
  if (active)
    for (int q = lane; q < n; q += 64) keys[wave][q] = edge_key(col[e0 + q], shift + 3 * (e0 + q));
  __syncthreads();
  uint64_t mine[kSortMax / 64];
  int rank[kSortMax / 64];
  if (active) {
    for (int t = 0; t < kSortMax / 64; ++t) {
      const int q = lane + 64 * t;
      if (q >= n) break;
      const uint64_t k = keys[wave][q];
      int rk = 0;
      for (int u = 0; u < n; ++u) rk += keys[wave][u] < k;
      mine[t] = k;
      rank[t] = rk;
    }
    for (int t = 0; t < kSortMax / 64; ++t) {
      const int q = lane + 64 * t;
      if (q >= n) break;
      const uint64_t k = mine[t];
      const int64_t e = e0 + rank[t];
      col[e] = (int32_t)(k >> 24);
      shift[3 * e] = (int8_t)((int)((k >> 16) & 255) - 128);
      shift[3 * e + 1] = (int8_t)((int)((k >> 8) & 255) - 128);
      shift[3 * e + 2] = (int8_t)((int)(k & 255) - 128);
    }
  }
}

// rev[e] of every edge e = (i, j, n): the slot of (j, i, -n) in row j (a
// binary search of the sorted row).  One group of kRevLanes lanes per row i.
constexpr int kRevLanes = 16;
__global__ void __launch_bounds__(256) k_rev(const int64_t* __restrict__ row_ptr, int64_t N, int64_t capacity,
                                             const int32_t* __restrict__ col, const int8_t* __restrict__ shift,
                                             int32_t* __restrict__ rev, int32_t* status) {
  const int64_t E = row_ptr[N];
  if (E > capacity) return;
  const int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kRevLanes;
  if (row >= N) return;
  const int32_t i = (int32_t)row;
  for (int64_t e = row_ptr[i] + threadIdx.x % kRevLanes; e < row_ptr[i + 1]; e += kRevLanes) {
    const int32_t j = col[e];
    const int8_t nn[3] = {(int8_t)-shift[3 * e], (int8_t)-shift[3 * e + 1], (int8_t)-shift[3 * e + 2]};
    const uint64_t want = edge_key(i, nn);
    int64_t a = row_ptr[j], b = row_ptr[j + 1];   // search [a, b)
    int32_t found = -1;
    while (a < b) {
      int64_t mid = (a + b) >> 1;
      uint64_t k = edge_key(col[mid], shift + 3 * mid);
      if (k == want) { found = (int32_t)mid; break; }
      if (k < want) a = mid + 1; else b = mid;
    }
    rev[e] = found;
    if (found < 0) atomicOr(status, AFM_FLAG_CAPACITY);
  }
}

// ---- exclusive scan (two levels, 1024 elements per block) ----
template <class T>
__global__ void __launch_bounds__(256) k_scan_blocks(const T* __restrict__ in, T* __restrict__ out,
                                                     int64_t n, T* __restrict__ sums) {
  __shared__ T part[256];
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  T v[4];
  T loc = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = (base + q < n) ? in[base + q] : T(0);
    loc += v[q];
  }
  part[threadIdx.x] = loc;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    T t = threadIdx.x >= off ? part[threadIdx.x - off] : T(0);
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  T run = part[threadIdx.x] - loc;
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

template <class T>
__global__ void __launch_bounds__(1024) k_scan_sums(T* sums, int64_t nb) {
  __shared__ T part[1024];
  T carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t q = c0 + threadIdx.x;
    T v = q < nb ? sums[q] : T(0);
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      T t = threadIdx.x >= off ? part[threadIdx.x - off] : T(0);
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (q < nb) sums[q] = carry + part[threadIdx.x] - v;
    T tot = part[1023];
    __syncthreads();
    carry += tot;
  }
}

template <class T>
__global__ void k_scan_add(T* __restrict__ out, int64_t n, const T* __restrict__ sums) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) out[q] += sums[q / 1024];
}

template <class T>
static int exclusive_scan(const T* in, T* out, int64_t n, T* sums, hipStream_t st) {
  if (n <= 0) return AFM_OK;
  const int64_t nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3((unsigned)nb), dim3(256), 0, st, in, out, n, sums);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(1024), 0, st, sums, nb);
  hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n,
                     (const T*)sums);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

__global__ void k_copy_count(const int64_t* row_ptr, int64_t N, int64_t* n_edges) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *n_edges = row_ptr[N];
}

__global__ void k_capacity_flag(const int64_t* row_ptr, int64_t N, int64_t capacity, int32_t* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && row_ptr[N] > capacity) atomicOr(status, AFM_FLAG_CAPACITY);
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

// ---- restriction to the cutoff: one wavefront per row ----
// flag[e] = |delta_e| < r_cut (the geometry kernel's arithmetic); cnt[i] =
// active edges of row i.  Nothing is written if the list overflowed.
__global__ void __launch_bounds__(256) k_active_rows(const int64_t* __restrict__ row_ptr, int64_t N,
                                                     int64_t capacity, const double* __restrict__ pos,
                                                     const double* __restrict__ cell,
                                                     const uint8_t* __restrict__ pbc,
                                                     const int64_t* __restrict__ seg, int64_t B,
                                                     const int32_t* __restrict__ col,
                                                     const int8_t* __restrict__ shift, float r_cut,
                                                     uint8_t* __restrict__ flag, int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i > N) return;
  if (row_ptr[N] > capacity) return;
  if (i == N) {
    if (lane == 0) cnt[N] = 0;
    return;
  }
  const int64_t sl = struct_of(seg, B, i);
  const bool per = pbc[sl] != 0;
  int n = 0;
  for (int64_t e = row_ptr[i] + lane; e < row_ptr[i + 1]; e += 64) {
    float dx, dy, dz;
    edge_vec_f32(pos, cell, per, sl, i, col[e], shift + 3 * e, dx, dy, dz);
    const bool act = edge_norm_f32(dx, dy, dz) / r_cut < 1.0f;
    flag[e] = act ? 1 : 0;
    n += act ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if (lane == 0) cnt[i] = n;
}

// compacted col/shift in row order; map[c] = listed edge, idx[e] = its slot
__global__ void __launch_bounds__(256) k_compact_rows(const int64_t* __restrict__ row_ptr, int64_t N,
                                                      int64_t capacity, const int64_t* __restrict__ crow,
                                                      const uint8_t* __restrict__ flag,
                                                      const int32_t* __restrict__ col,
                                                      const int8_t* __restrict__ shift, int32_t* __restrict__ ccol,
                                                      int8_t* __restrict__ cshift, int32_t* __restrict__ map,
                                                      int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  if (row_ptr[N] > capacity) return;
  int64_t base = crow[i];
  for (int64_t e0 = row_ptr[i]; e0 < row_ptr[i + 1]; e0 += 64) {
    const int64_t e = e0 + lane;
    const bool act = e < row_ptr[i + 1] && flag[e];
    const uint64_t m = __ballot(act);
    if (act) {
      const int64_t c = base + __popcll(m & ((uint64_t(1) << lane) - 1));
      ccol[c] = col[e];
      cshift[3 * c] = shift[3 * e];
      cshift[3 * c + 1] = shift[3 * e + 1];
      cshift[3 * c + 2] = shift[3 * e + 2];
      map[c] = (int32_t)e;
      idx[e] = (int32_t)c;
    }
    base += __popcll(m);
  }
}

// rev of a kept edge is kept (delta_rev = -delta_e bit for bit, so the
// norms agree); the flag test only guards the index
__global__ void k_compact_rev(const int64_t* __restrict__ row_ptr, int64_t N, int64_t capacity,
                              const int64_t* __restrict__ crow, const int32_t* __restrict__ map,
                              const int32_t* __restrict__ rev, const uint8_t* __restrict__ flag,
                              const int32_t* __restrict__ idx, int32_t* __restrict__ crev,
                              int64_t* __restrict__ n_edges) {
  if (row_ptr[N] > capacity) return;
  const int64_t E = crow[N];
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_edges = E;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < E; c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = rev[map[c]];
    crev[c] = flag[r] ? idx[r] : (int32_t)c;
  }
}

int launch_compact_to_cutoff(const SysDev& s, const NlDev& in, float r_cut, const afm_workspace* ws,
                             const WsLayout& L, NlDev* out, hipStream_t st) {
  TraceScope tr(st, "compact");
  const int64_t N = s.N;
  int64_t* crow = ws_ptr<int64_t>(ws, L.c_row_ptr);
  uint8_t* flag = ws_ptr<uint8_t>(ws, L.c_flag);
  int64_t* cnt = ws_ptr<int64_t>(ws, L.nb_counts);
  int64_t* sums = ws_ptr<int64_t>(ws, L.nb_scan);
  NlDev o = in;
  o.row_ptr = crow;
  o.col = ws_ptr<int32_t>(ws, L.c_col);
  o.shift = ws_ptr<int8_t>(ws, L.c_shift);
  o.rev = ws_ptr<int32_t>(ws, L.c_rev);
  o.n_edges = ws_ptr<int64_t>(ws, L.c_n_edges);
  // an overflowed list leaves an empty compacted list (the status flag is set)
  int rc = zero_async(crow, (N + 1) * 8, st);
  if (!rc) rc = zero_async(cnt, (N + 1) * 8, st);
  if (rc) return rc;
  if (in.capacity > 0) {
    hipLaunchKernelGGL(k_active_rows, dim3(nblk(N + 1, 4)), dim3(256), 0, st, (const int64_t*)in.row_ptr, N,
                       in.capacity, s.pos, s.cell, s.pbc, s.seg, s.B, (const int32_t*)in.col,
                       (const int8_t*)in.shift, r_cut, flag, cnt);
    rc = exclusive_scan<int64_t>(cnt, crow, N + 1, sums, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_compact_rows, dim3(nblk(N, 4)), dim3(256), 0, st, (const int64_t*)in.row_ptr, N,
                       in.capacity, (const int64_t*)crow, (const uint8_t*)flag, (const int32_t*)in.col,
                       (const int8_t*)in.shift, o.col, o.shift, ws_ptr<int32_t>(ws, L.c_map),
                       ws_ptr<int32_t>(ws, L.c_idx));
    hipLaunchKernelGGL(k_compact_rev, dim3(2048), dim3(256), 0, st, (const int64_t*)in.row_ptr, N, in.capacity,
                       (const int64_t*)crow, (const int32_t*)ws_ptr<int32_t>(ws, L.c_map),
                       (const int32_t*)in.rev, (const uint8_t*)flag, (const int32_t*)ws_ptr<int32_t>(ws, L.c_idx),
                       o.rev, o.n_edges);
  }
  AFM_LAUNCH_CHECK();
  *out = o;
  return AFM_OK;
}

int launch_build_neighbors(const SysDev& s, double r_list, const NlDev& nl, const afm_workspace* ws,
                           const WsLayout& L, int n_species, hipStream_t st) {
  const int64_t N = s.N, B = s.B;
  StructMeta* meta = ws_ptr<StructMeta>(ws, L.nb_struct);
  AtomMeta* am = ws_ptr<AtomMeta>(ws, L.nb_atom);
  int32_t* bcount = ws_ptr<int32_t>(ws, L.nb_bin_count);
  int32_t* bstart = ws_ptr<int32_t>(ws, L.nb_bin_start);
  int32_t* batoms = ws_ptr<int32_t>(ws, L.nb_bin_atoms);
  int64_t* counts = ws_ptr<int64_t>(ws, L.nb_counts);
  int64_t* sums = ws_ptr<int64_t>(ws, L.nb_scan);
  const double r2 = r_list * r_list;
  TraceScope tr(st, "neighbors");
  int rc0 = zero_async(bcount, (L.n_bins_max + 1) * 4, st);
  if (rc0) return rc0;
  hipLaunchKernelGGL(k_struct_prep, dim3(nblk(B, 64)), dim3(64), 0, st, s.cell, s.pbc, s.seg, B, r_list,
                     meta, nl.status);
  hipLaunchKernelGGL(k_bin_offsets, dim3(1), dim3(1), 0, st, meta, B);
  hipLaunchKernelGGL(k_atom_prep, dim3(nblk(N, 256)), dim3(256), 0, st, s.pos, s.species, s.pbc, s.seg, N,
                     B, n_species, (const StructMeta*)meta, am, bcount, nl.status);
  AFM_LAUNCH_CHECK();
  // bstart[b] = first slot of bin b, bstart[n_bins_max] = total
  int rc = exclusive_scan<int32_t>(bcount, bstart, L.n_bins_max + 1, reinterpret_cast<int32_t*>(sums), st);
  if (rc) return rc;
  // bcount becomes the fill cursor
  rc = zero_async(bcount, (L.n_bins_max + 1) * 4, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_bin_fill, dim3(nblk(N, 256)), dim3(256), 0, st, (const AtomMeta*)am, N,
                     (const int32_t*)bstart, bcount, batoms);
  AFM_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rows<false>, dim3(nblk(N + 1, 4)), dim3(256), 0, st, s.pos, s.cell, s.pbc, s.seg,
                     N, B, r2, (const StructMeta*)meta, (const AtomMeta*)am, (const int32_t*)bstart,
                     (const int32_t*)batoms, counts, (const int64_t*)nullptr,
                     nl.capacity, nl.col, nl.shift, nl.status, (int)ws->max_row);
  AFM_LAUNCH_CHECK();
  rc = exclusive_scan<int64_t>(counts, nl.row_ptr, N + 1, sums, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(1), 0, st, (const int64_t*)nl.row_ptr, N, nl.n_edges);
  hipLaunchKernelGGL(k_capacity_flag, dim3(1), dim3(1), 0, st, (const int64_t*)nl.row_ptr, N, nl.capacity,
                     nl.status);
  hipLaunchKernelGGL(k_rows<true>, dim3(nblk(N, 4)), dim3(256), 0, st, s.pos, s.cell, s.pbc, s.seg, N, B,
                     r2, (const StructMeta*)meta, (const AtomMeta*)am, (const int32_t*)bstart,
                     (const int32_t*)batoms, counts, (const int64_t*)nl.row_ptr,
                     nl.capacity, nl.col, nl.shift, nl.status, (int)ws->max_row);
  hipLaunchKernelGGL(k_row_sort, dim3(nblk(N, 4)), dim3(256), 0, st, s.seg, N, B, (const StructMeta*)meta,
                     (const int64_t*)nl.row_ptr, nl.capacity, nl.col, nl.shift);
  hipLaunchKernelGGL(k_rev, dim3(nblk(N, 256 / kRevLanes)), dim3(256), 0, st, (const int64_t*)nl.row_ptr, N,
                     nl.capacity, (const int32_t*)nl.col, (const int8_t*)nl.shift, nl.rev, nl.status);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

// chunk c covers rows [a_c, a_{c+1}) with a_c the first row starting at or
// after c * chunk_edges; a_{n_chunks} = N.
__global__ void k_chunk_rows(const int64_t* __restrict__ row_ptr, int64_t N, int64_t ce, int64_t nc,
                             int64_t* __restrict__ out) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c > nc) return;
  if (c == nc) { out[c] = N; return; }
  const int64_t target = c * ce;
  int64_t lo = 0, hi = N + 1;   // first index with row_ptr[idx] >= target
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (row_ptr[mid] >= target) hi = mid; else lo = mid + 1;
  }
  out[c] = lo > N ? N : lo;
}

// Every chunk must fit the chunk buffers; otherwise (or if the list itself
// overflowed) all chunks are emptied and AFM_FLAG_CAPACITY is set, so no
// later kernel reads past a buffer.
__global__ void k_check_chunks(const int64_t* __restrict__ row_ptr, int64_t N, int64_t capacity, int64_t cex,
                               int64_t nc, int64_t* __restrict__ cr, int32_t* status) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  bool bad = row_ptr[N] > capacity;
  for (int64_t c = 0; c < nc && !bad; ++c) bad = (row_ptr[cr[c + 1]] - row_ptr[cr[c]]) > cex;
  if (bad) {
    for (int64_t c = 0; c <= nc; ++c) cr[c] = 0;
    atomicOr(status, AFM_FLAG_CAPACITY);
  }
}

int check_chunks(const SysDev& s, const NlDev& nl, const afm_workspace* ws, const WsLayout& L, hipStream_t st) {
  hipLaunchKernelGGL(k_check_chunks, dim3(1), dim3(1), 0, st, (const int64_t*)nl.row_ptr, s.N, nl.capacity, L.cex,
                     ws->n_chunks, ws_ptr<int64_t>(ws, L.chunk_rows), nl.status);
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

int launch_chunk_rows(const SysDev& s, const NlDev& nl, const afm_workspace* ws, const WsLayout& L,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_rows, dim3(nblk(ws->n_chunks + 1, 64)), dim3(64), 0, st,
                     (const int64_t*)nl.row_ptr, s.N, ws->chunk_edges, ws->n_chunks,
                     ws_ptr<int64_t>(ws, L.chunk_rows));
  AFM_LAUNCH_CHECK();
  return AFM_OK;
}

}  // namespace afm
