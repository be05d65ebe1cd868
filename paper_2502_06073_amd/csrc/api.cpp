// C ABI entry points: argument checks and the chunk schedule.
#include <cmath>
#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"

namespace afm {

static int check_sys(const afm_system* sys, const afm_workspace* ws, SysDev* out) {
  if (!sys || !ws) { set_error("null system or workspace"); return AFM_E_INVALID; }
  if (!sys->pos || !sys->species || !sys->cell || !sys->pbc || !sys->seg) {
    set_error("null system array"); return AFM_E_INVALID;
  }
  if (sys->n_atoms != ws->n_atoms || sys->n_struct != ws->n_struct) {
    set_error("system sizes differ from the workspace plan"); return AFM_E_INVALID;
  }
  if (!ws->ptr) { set_error("workspace pointer is null"); return AFM_E_INVALID; }
  out->N = sys->n_atoms; out->B = sys->n_struct; out->pos = sys->pos; out->species = sys->species;
  out->cell = sys->cell; out->pbc = sys->pbc; out->seg = sys->seg;
  return AFM_OK;
}

static int check_nl(const afm_nlist* nl, const afm_workspace* ws, NlDev* out) {
  if (!nl || !nl->row_ptr || !nl->n_edges || !nl->status) { set_error("null neighbour-list array"); return AFM_E_INVALID; }
  if (nl->capacity > 0 && (!nl->col || !nl->shift || !nl->rev)) { set_error("null neighbour-list array"); return AFM_E_INVALID; }
  if (nl->capacity > ws->edge_capacity) { set_error("neighbour-list capacity exceeds the workspace plan"); return AFM_E_INVALID; }
  out->capacity = nl->capacity; out->row_ptr = nl->row_ptr; out->col = nl->col; out->shift = nl->shift;
  out->rev = nl->rev; out->n_edges = nl->n_edges; out->status = nl->status;
  return AFM_OK;
}

static int check_model(const afm_model* m, const afm_workspace* ws, WsLayout* L) {
  if (!m) { set_error("null model"); return AFM_E_INVALID; }
  if (ws->precision != m->prec) { set_error("workspace planned for another precision"); return AFM_E_INVALID; }
  *L = workspace_layout(m, ws);
  if (ws->bytes < L->total) { set_error("workspace smaller than its plan"); return AFM_E_CAPACITY; }
  return AFM_OK;
}

// energies, forces and virial for already-checked arguments (also used by md.hip)
int api_energy_forces_dev(const afm_model* m, const SysDev& s, const NlDev& n, double* e_atom, double* e_struct,
                          double* forces, double* virial, const afm_workspace* ws, const WsLayout& L,
                          hipStream_t st) {
  int rc = launch_chunk_rows(s, n, ws, L, st);
  if (!rc) rc = check_chunks(s, n, ws, L, st);
  const bool fused = m->fuse_last && mfma_fused_last_available(m);
  for (int c = 0; !rc && c < ws->n_chunks; ++c) {
    rc = run_forward_chunk(m, s, n, ws, L, c, st, fused);
    if (!rc) rc = run_backward_chunk(m, s, n, ws, L, c, nullptr, st, fused);
  }
  if (!rc) rc = run_atom_energy(m, s, n, ws, L, e_atom, e_struct, st);
  if (!rc && (forces || virial)) rc = run_force_scatter(m, s, n, ws, L, forces, virial, st);
  return rc;
}

}  // namespace afm

using namespace afm;

extern "C" {

int afm_build_neighbors(const afm_system* sys, double r_list, afm_nlist* nl, const afm_workspace* ws,
                        void* stream) {
  SysDev s{};
  NlDev n{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (rc) return rc;
  if (!(r_list > 0) || !(r_list < 1e4)) { set_error("r_list must be positive and finite"); return AFM_E_INVALID; }
  WsLayout L = workspace_layout(nullptr, ws);
  if (ws->bytes < L.total) { set_error("workspace smaller than its plan"); return AFM_E_CAPACITY; }
  return launch_build_neighbors(s, r_list, n, ws, L, kMaxSpecies * 1024, (hipStream_t)stream);
}

int afm_forward_energy(const afm_model* m, const afm_system* sys, const afm_nlist* nl, double* e_atom,
                       double* e_struct, const afm_workspace* ws, void* stream) {
  SysDev s{};
  NlDev n{};
  WsLayout L{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (!rc) rc = check_model(m, ws, &L);
  if (rc) return rc;
  if (!e_atom) { set_error("e_atom is required"); return AFM_E_INVALID; }
  hipStream_t st = (hipStream_t)stream;
  rc = launch_chunk_rows(s, n, ws, L, st);
  if (!rc) rc = check_chunks(s, n, ws, L, st);
  for (int c = 0; !rc && c < ws->n_chunks; ++c) rc = run_forward_chunk(m, s, n, ws, L, c, st);
  if (!rc) rc = run_atom_energy(m, s, n, ws, L, e_atom, e_struct, st);
  return rc;
}

int afm_backward_forces(const afm_model* m, const afm_system* sys, const afm_nlist* nl,
                        const double* grad_e_struct, double* forces, double* virial, const afm_workspace* ws,
                        void* stream) {
  SysDev s{};
  NlDev n{};
  WsLayout L{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (!rc) rc = check_model(m, ws, &L);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  for (int c = 0; !rc && c < ws->n_chunks; ++c) {
    // a single chunk keeps the forward state; several chunks recompute it
    if (ws->n_chunks > 1) rc = run_forward_chunk(m, s, n, ws, L, c, st);
    if (!rc) rc = run_backward_chunk(m, s, n, ws, L, c, grad_e_struct, st);
  }
  if (!rc && (forces || virial)) rc = run_force_scatter(m, s, n, ws, L, forces, virial, st);
  return rc;
}

int afm_energy_forces(const afm_model* m, const afm_system* sys, const afm_nlist* nl, double* e_atom,
                      double* e_struct, double* forces, double* virial, const afm_workspace* ws, void* stream) {
  SysDev s{};
  NlDev n{};
  WsLayout L{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (!rc) rc = check_model(m, ws, &L);
  if (rc) return rc;
  if (!e_atom) { set_error("e_atom is required"); return AFM_E_INVALID; }
  return api_energy_forces_dev(m, s, n, e_atom, e_struct, forces, virial, ws, L, (hipStream_t)stream);
}

int afm_backward_forces_backward(const afm_model* m, const afm_system* sys, const afm_nlist* nl,
                                 const double* grad_e_struct, const double* grad_forces,
                                 const double* grad_virial, float* grad_weights, double* grad_pos,
                                 const afm_workspace* ws, void* stream) {
  SysDev s{};
  NlDev n{};
  WsLayout L{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (!rc) rc = check_model(m, ws, &L);
  if (rc) return rc;
  if (!grad_weights) { set_error("grad_weights is required"); return AFM_E_INVALID; }
  if (!ws->with_second_order) { set_error("workspace was planned without the second-order buffers"); return AFM_E_INVALID; }
  return run_second_order(m, s, n, ws, L, grad_e_struct, grad_forces, grad_virial, grad_weights, grad_pos,
                          (hipStream_t)stream);
}

int afm_md_step(const afm_model* m, const afm_system* sys, afm_nlist* nl, afm_md_state* state, int32_t n_steps,
                const afm_workspace* ws, void* stream) {
  SysDev s{};
  NlDev n{};
  WsLayout L{};
  int rc = check_sys(sys, ws, &s);
  if (!rc) rc = check_nl(nl, ws, &n);
  if (!rc) rc = check_model(m, ws, &L);
  if (rc) return rc;
  if (!state || !state->pos || !state->vel || !state->forces || !state->mass_by_species || !state->energy_log ||
      !state->e_atom || !state->e_struct) {
    set_error("null MD state array");
    return AFM_E_INVALID;
  }
  if (n_steps < 0 || !(state->dt_fs > 0) || !(state->skin >= 0) || state->rebuild_every < 0 || state->step < 0) {
    set_error("bad MD parameters");
    return AFM_E_INVALID;
  }
  if (state->t_target_K > 0 && (!(state->tau_fs > 0) || !std::isfinite(state->t_target_K) || !state->nh)) {
    set_error("NVT needs tau_fs > 0, a finite target temperature and the thermostat state array");
    return AFM_E_INVALID;
  }
  s.pos = state->pos;
  return md_step(m, s, n, state, n_steps, ws, L, (hipStream_t)stream);
}

}  // extern "C"
