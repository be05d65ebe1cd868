// Packs the flat float64 weight vector into the device layouts the kernels
// read (one device allocation per model).
#include <hip/hip_runtime.h>
#include <string.h>

#include <string>
#include <vector>

#include "internal.h"

namespace afm {
void pack_bf16_frags(const afm_model* m, const double* w, std::vector<char>& out, DevWeights* Wd);  // mfma_chain.hip
int mfma_check_shape(const afm_model* m);                                                         // mfma_chain.hip
}

namespace afm {

// float -> bf16 bits, rounding to nearest even (weights are finite)
static uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static float bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

static const afm_param_block* find_block(const afm_model* m, const char* name) {
  for (auto& b : m->blocks)
    if (strcmp(b.name, name) == 0) return &b;
  return nullptr;
}

int pack_weights(afm_model* m, const double* w) {
  const ModelDims& d = m->dims;
  std::vector<char> host;
  auto reserve = [&](int64_t bytes) {
    int64_t o = (int64_t)host.size();
    int64_t pad = (bytes + 255) & ~int64_t(255);
    host.resize(o + pad, 0);
    return o;
  };
  struct Fix { const void** dst; int64_t off; };
  std::vector<Fix> fix;
  auto put_f32 = [&](const void** dst, const double* src, int64_t n) {
    int64_t o = reserve(n * 4);
    float* p = reinterpret_cast<float*>(host.data() + o);
    for (int64_t q = 0; q < n; ++q) p[q] = (float)src[q];
    fix.push_back({dst, o});
  };
  char nm[32];
  if (m->prec == AFM_BF16_MFMA) {
    int rc = mfma_check_shape(m);
    if (rc) return rc;
  }

  for (int k = 0; k < d.ntb; ++k) {
    snprintf(nm, sizeof nm, "twobody.%d", k);
    const afm_param_block* b = find_block(m, nm);
    put_f32((const void**)&m->W.tb[k], w + b->offset, b->rows * b->cols);
  }
  for (int L = 1; L <= d.NL; ++L) {
    snprintf(nm, sizeof nm, "layer%d.env", L);
    const afm_param_block* b = find_block(m, nm);
    std::vector<double> perm((size_t)b->rows * b->cols);
    for (int l = 0; l <= d.lmax; ++l)
      for (int n = 0; n < d.c; ++n)
        memcpy(&perm[((size_t)l * d.c + n) * d.w], w + b->offset + ((size_t)n * (d.lmax + 1) + l) * d.w,
               sizeof(double) * d.w);
    put_f32((const void**)&m->W.env[L - 1], perm.data(), (int64_t)perm.size());
    for (int k = 0; k < d.depth; ++k) {
      snprintf(nm, sizeof nm, "layer%d.latent.%d", L, k);
      b = find_block(m, nm);
      put_f32((const void**)&m->W.lat[L - 1][k], w + b->offset, b->rows * b->cols);
    }
    if (L < d.NL && d.dense) {
      // regroup the per-path matrices by output irrep: A_r = [A_k1 | A_k2 | ...]
      snprintf(nm, sizeof nm, "layer%d.mix", L);
      b = find_block(m, nm);
      const LayerPlan& lp = m->plan.layer[L - 1];
      std::vector<double> rep;
      for (int r = 0; r < lp.n_out; ++r) {
        m->W.mix_off[L - 1][r] = (int64_t)rep.size();
        std::vector<int> ks;
        for (int k = 0; k < lp.n_paths; ++k)
          if (lp.p[k].out_off == lp.out_off[r]) ks.push_back(k);
        const size_t np = ks.size(), o = rep.size();
        rep.resize(o + np * d.c * d.c);
        for (int n = 0; n < d.c; ++n)
          for (size_t j = 0; j < np; ++j)
            memcpy(&rep[o + ((size_t)n * np + j) * d.c], w + b->offset + ((size_t)ks[j] * d.c + n) * d.c,
                   sizeof(double) * d.c);
      }
      put_f32((const void**)&m->W.mix[L - 1], rep.data(), (int64_t)rep.size());
      if (m->prec == AFM_BF16_MFMA) {
        // hi = bf16(f), lo = bf16(f - hi) of the FP32 value f, for A_r and A_r^T
        const int64_t T = (int64_t)rep.size();
        m->W.mix_elems[L - 1] = T;
        int64_t o = reserve(4 * T * 2);
        uint16_t* q = reinterpret_cast<uint16_t*>(host.data() + o);
        auto split = [&](int64_t dst, double v) {
          const float f = (float)v;
          const uint16_t h = bf16_rne(f);
          q[dst] = h;
          q[T + dst] = bf16_rne(f - bf16_value(h));
        };
        for (int r = 0; r < lp.n_out; ++r) {
          int np = 0;
          for (int k = 0; k < lp.n_paths; ++k) np += lp.p[k].out_off == lp.out_off[r];
          const int64_t base = m->W.mix_off[L - 1][r], K = (int64_t)np * d.c;
          for (int64_t n = 0; n < d.c; ++n)
            for (int64_t k = 0; k < K; ++k) {
              split(base + n * K + k, rep[base + n * K + k]);
              split(2 * T + base + k * d.c + n, rep[base + n * K + k]);
            }
        }
        fix.push_back({(const void**)&m->W.mix_b16[L - 1], o});
      }
    } else if (L < d.NL) {
      snprintf(nm, sizeof nm, "layer%d.alpha", L);
      b = find_block(m, nm);
      put_f32((const void**)&m->W.alpha[L - 1], w + b->offset, b->rows * b->cols);
    }
  }
  const afm_param_block* e0 = find_block(m, "edge.0");
  const afm_param_block* e1 = find_block(m, "edge.1");
  put_f32((const void**)&m->W.e0, w + e0->offset, e0->rows * e0->cols);
  put_f32((const void**)&m->W.e1, w + e1->offset, e1->rows * e1->cols);
  std::vector<double> weff(d.w, 0.0);
  for (int hh = 0; hh < d.h; ++hh) {
    double a = w[e1->offset + hh];
    for (int f = 0; f < d.w; ++f) weff[f] += w[e0->offset + (int64_t)hh * d.w + f] * a;
  }
  put_f32((const void**)&m->W.w_eff, weff.data(), d.w);
  {
    const afm_param_block* sc = find_block(m, "species.scale");
    const afm_param_block* sh = find_block(m, "species.shift");
    int64_t o = reserve(d.S * 8);
    memcpy(host.data() + o, w + sc->offset, d.S * 8);
    fix.push_back({(const void**)&m->W.sp_scale, o});
    o = reserve(d.S * 8);
    memcpy(host.data() + o, w + sh->offset, d.S * 8);
    fix.push_back({(const void**)&m->W.sp_shift, o});
  }
  int64_t frag_off = -1;
  if (m->prec == AFM_BF16_MFMA) {
    std::vector<char> frags;
    pack_bf16_frags(m, w, frags, &m->W);
    frag_off = reserve((int64_t)frags.size());
    memcpy(host.data() + frag_off, frags.data(), frags.size());
  }
  // a repack (new weight values, same model) reuses the allocation: the
  // layout depends only on the shapes
  void* dev = m->dev_mem;
  hipError_t e = hipSuccess;
  if (dev && m->dev_bytes != (int64_t)host.size()) { set_error("internal: weight layout changed"); return AFM_E_INVALID; }
  if (!dev) {
    e = hipMalloc(&dev, host.size());
    if (e != hipSuccess) { set_error(std::string("hipMalloc weights: ") + hipGetErrorString(e)); return AFM_E_HIP; }
    m->dev_mem = dev;
    m->dev_bytes = (int64_t)host.size();
  }
  e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { set_error(std::string("hipMemcpy weights: ") + hipGetErrorString(e)); return AFM_E_HIP; }
  for (auto& f : fix) *f.dst = static_cast<char*>(dev) + f.off;
  if (frag_off >= 0) m->W.frag = static_cast<char*>(dev) + frag_off;
  return AFM_OK;
}

}  // namespace afm
