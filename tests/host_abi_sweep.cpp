// Host-only sweep of the C ABI's entry points that make no GPU call (weight
// layout, real CG tensors, stage costs, workspace planning) over a grid of
// hyperparameters, built with AddressSanitizer on the host code: an
// out-of-bounds host write in any of them fails the run.
#include <cstdio>
#include <cstring>
#include <vector>
#include "afm.h"
int main() {
  int n_ok = 0, n_err = 0;
  for (int lmax = 0; lmax <= 3; ++lmax)
    for (int NL = 1; NL <= 3; ++NL)
      for (int c : {8, 16, 32, 64, 128})
        for (int mixing = 0; mixing <= 1; ++mixing)
          for (int w : {32, 64, 256, 512}) {
            afm_hparams h{};
            h.n_species = 4; h.l_max = lmax; h.n_layers = NL; h.latent = w; h.channels = c;
            h.n_bessel = 8; h.poly_p = 6; h.n_twobody = 3; h.twobody[0] = w / 4; h.twobody[1] = w / 2;
            h.twobody[2] = w; h.latent_depth = 3; h.edge_hidden = 16; h.r_cut = 5.0;
            h.avg_num_neighbors = 30; h.energy_scale = 1; h.mixing = mixing;
            int64_t nb = 0, np = 0;
            int rc = afm_param_layout_size(&h, &nb, &np);
            if (rc) { ++n_err; continue; }
            for (int64_t k = 0; k < nb; ++k) { afm_param_block b; afm_param_layout_block(&h, k, &b); }
            afm_stage_cost sc[64]; int32_t ns = 0;
            rc = afm_stage_costs(&h, sc, 64, &ns);
            if (rc || ns > 64) { printf("stage costs rc %d n %d\n", rc, ns); return 1; }
            ++n_ok;
          }
  for (int l1 = 0; l1 <= 3; ++l1)
    for (int l2 = 0; l2 <= 3; ++l2)
      for (int l3 = 0; l3 <= 6; ++l3) {
        std::vector<double> out(7 * 7 * 13);
        afm_cg_real(l1, l2, l3, out.data());
      }
  afm_workspace ws;
  afm_workspace_plan(nullptr, 1000, 4, 50000, 0, 0, &ws);
  printf("ok %d refused %d\n", n_ok, n_err);
  return 0;
}
