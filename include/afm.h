/*
 * afm.h -- C ABI of the MI355X (gfx950) library for the strictly-local
 * E(3)-equivariant edge potential trained as Allegro-FM (arXiv 2502.06073).
 *
 * The library computes, on one GPU, energies and their derivatives for
 * atoms that interact only within a radial cutoff (the "strictly-local"
 * architecture of the paper's Abstract; its hyperparameters are given in
 * Methodology / Model Training and Table 1):
 *
 *   edges     every ordered pair (i, j, n) with |r_j - r_i + n.h| < r_list,
 *             all periodic images n, canonical order (i, j, n0, n1, n2);
 *   basis     n_b Bessel functions times a polynomial cutoff envelope of the
 *             edge length; real spherical harmonics (l <= l_max) of its
 *             direction;
 *   network   two-body latent MLP -> per-layer linear environment embedding,
 *             environment sum over the central atom's edges, channelwise
 *             Clebsch-Gordan tensor products, latent MLP with residual ->
 *             linear edge-energy MLP;
 *   energies  E_i = sigma_Z * energy_scale * sum_{row i} eps_e + mu_Z,
 *             E_s = sum_{i in s} E_i;
 *   forces    F_i = -dE/dr_i = sum_{e in row i} (g_e - g_rev(e)) with
 *             g_e = dE/d(delta_e); virial W_s = -sum_{e in s} g_e delta_e^T.
 *
 * Conventions shared by every entry point
 *   - Pointers named in afm_system / afm_nlist and every per-atom or
 *     per-structure output are DEVICE pointers owned by the caller.  The
 *     library never frees them.  Host pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued asynchronously on it; no entry point
 *     allocates device memory or synchronises the stream except
 *     afm_model_create / afm_model_destroy.
 *   - Units: Angstrom, eV, amu, fs.  Cells are row-major [3][3] with the
 *     lattice vectors a, b, c as rows; a structure is either periodic in all
 *     three directions (pbc = 1) or open (pbc = 0).  Positions are used as
 *     given (never wrapped by the evaluation calls).
 *   - Return value: AFM_OK (0) or a negative afm_status.  Nothing throws
 *     across the ABI.  afm_last_error() gives a message for the calling
 *     thread.  Conditions found on the device (edge capacity overflow,
 *     non-finite positions, species out of range, MD skin violation) are
 *     OR-ed into the device word nlist->status; the caller reads it when it
 *     synchronises.
 */
#ifndef AFM_H_
#define AFM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef enum {
  AFM_OK = 0,
  AFM_E_INVALID = -1,     /* null pointer, bad size or hyperparameter       */
  AFM_E_CAPACITY = -2,    /* a caller buffer is too small                   */
  AFM_E_NONFINITE = -3,   /* non-finite input found on the host             */
  AFM_E_UNSUPPORTED = -4, /* precision or shape not built into this library */
  AFM_E_HIP = -5,         /* HIP runtime error (see afm_last_error)         */
  AFM_E_WEIGHTS = -6      /* weight vector length does not match layout     */
} afm_status;

/* bits of the device status word nlist->status */
#define AFM_FLAG_CAPACITY 1   /* edges exceeded nlist->capacity; n_edges holds the need */
#define AFM_FLAG_NONFINITE 2  /* a position was not finite                               */
#define AFM_FLAG_SPECIES 4    /* a species index was outside [0, n_species)              */
#define AFM_FLAG_SKIN 8       /* an atom moved more than skin/2 since the last rebuild    */
#define AFM_FLAG_IMAGES 16    /* a periodic image index did not fit in int8               */

typedef enum {
  AFM_FP64_REF = 0,    /* not built: the FP64 reference is the CPU oracle     */
  AFM_FP32_PLAIN = 1,  /* every step in FP32 on the vector ALUs               */
  AFM_BF16_MFMA = 2,   /* MLP GEMMs on BF16 MFMA with FP32 accumulation       */
  AFM_BF16_MFMA_FAST_ADJOINT = 3
  /* as AFM_BF16_MFMA, but the adjoint (force) GEMMs use only the leading
   * bf16 term of each weight where the energy uses two: faster forces with
   * a larger error (still within the BF16 force tolerance) that are no
   * longer the exact gradient of the reported energy, so NVE energy
   * conservation degrades; workspaces are planned as for AFM_BF16_MFMA */
} afm_precision;

/* ---- hyperparameters (host struct) --------------------------------------
 * Methodology / Model Training and Table 1: tensor features `channels` with
 * l <= l_max in full O(3); two-body latent MLP widths twobody[0..n_twobody-1]
 * (the last equals `latent`); latent MLPs of depth latent_depth and width
 * `latent`; SiLU nonlinearities; edge-energy MLP latent -> edge_hidden -> 1
 * without nonlinearity; radial cutoff r_cut.  n_bessel radial functions with
 * a polynomial envelope of power poly_p; avg_num_neighbors normalises the
 * environment sum by its inverse square root. */
typedef struct {
  int32_t n_species;
  int32_t l_max;          /* 0..3 (3: one or two layers, 16 or 64 channels) */
  int32_t n_layers;       /* >= 1 */
  int32_t latent;         /* latent width w (multiple of 16) */
  int32_t channels;       /* tensor channels c: 8, 16, 32, 64 or 128 */
  int32_t n_bessel;       /* <= 16 */
  int32_t poly_p;         /* envelope power p >= 2 */
  int32_t n_twobody;      /* 1..4 */
  int32_t twobody[4];
  int32_t latent_depth;   /* 1..4 */
  int32_t edge_hidden;
  double r_cut;
  double avg_num_neighbors;
  double energy_scale;
  /* Mixing of the tensor-product outputs into the next layer's features
   * (Methodology / Model Training gives no equation for it):
   *   0 = one weight per (path, channel), alpha (default; the reading whose
   *       parameter counts are closest to Table 1);
   *   1 = dense: a channels x channels matrix per path (the alternative
   *       reading), built for l_max <= 2 and channels <= 64; the double
   *       backward refuses it. */
  int32_t mixing;
} afm_hparams;

/* ---- weight layout ------------------------------------------------------
 * The weights are one flat float64 vector made of these blocks in order
 * (matrices row-major, out x in):
 *   twobody.k           [twobody[k], k ? twobody[k-1] : 2 S + n_bessel]
 *   layerL.env          [channels * (l_max + 1), latent]   (row n*(l_max+1)+l)
 *   layerL.latent.k     [latent, k ? latent : latent + n0e_L * channels]
 *   layerL.alpha        [n_paths_L, channels]      (only for L < n_layers,
 *                                                    mixing = 0)
 *   layerL.mix          [n_paths_L * channels, channels]  (only for
 *                       L < n_layers, mixing = 1; row k*channels + n, column
 *                       m: output channel n of path k takes A_k[n][m] times
 *                       the path's input channel m)
 *   edge.0              [edge_hidden, latent]
 *   edge.1              [1, edge_hidden]
 *   species.scale       [S]       species.shift [S]
 * with n0e_L the number of tensor-product paths of layer L ending in a 0e
 * scalar.  `init` says how the seeded generator fills a block:
 *   0 = N(0, 1/fan_in), 1 = N(0, 1), 2 = ones. */
typedef struct {
  char name[32];
  int64_t offset;
  int64_t rows, cols;     /* cols = 1 for vectors */
  int64_t fan_in;
  int32_t init;
} afm_param_block;

/* Number of blocks and total parameter count for `hp`. */
int afm_param_layout_size(const afm_hparams* hp /*host*/, int64_t* n_blocks /*host*/,
                          int64_t* n_params /*host*/);
/* Block `k` (0-based) of the layout. */
int afm_param_layout_block(const afm_hparams* hp /*host*/, int64_t k,
                           afm_param_block* out /*host*/);

/* Real Clebsch-Gordan tensor C^{l1 l2 l3}[m1][m2][m3] as used by the
 * library (real spherical harmonics without Condon-Shortley phase, order
 * m = -l..l, l = 1 as (y, z, x); sum C^2 = 2 l3 + 1; first nonzero entry in
 * row-major order positive).  out: host, (2l1+1)(2l2+1)(2l3+1) doubles. */
int afm_cg_real(int32_t l1, int32_t l2, int32_t l3, double* out /*host*/);

/* ---- model --------------------------------------------------------------- */
typedef struct afm_model afm_model;

/* Copy `weights` (host, float64, afm_param_layout_size values) to the
 * device in the layouts the kernels of `precision` read.  Allocates device
 * memory owned by the model (freed by afm_model_destroy).  Synchronous. */
int afm_model_create(const afm_hparams* hp /*host*/, const double* weights /*host*/,
                     int64_t n_weights, afm_precision precision, afm_model** out /*host*/);
int afm_model_destroy(afm_model* model);

/* Replace the model's weight values (host, float64, the same layout and
 * count as at creation) — a training step's update.  Repacks into the
 * existing device allocation after a device-wide synchronisation, so no
 * work that reads the model may be in flight or captured in a graph being
 * replayed; blocking; allocates nothing. */
int afm_model_set_weights(afm_model* model, const double* weights /*host*/, int64_t n_weights);

/* One Adam update (Model Training: parameters optimised with Adam; Kingma &
 * Ba's algorithm with bias correction): for q < n,
 *   m1 = b1 m1 + (1 - b1) g;  m2 = b2 m2 + (1 - b2) g^2;
 *   theta -= lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps)
 * with g = grad[q] (float32, e.g. afm_backward_forces_backward's output)
 * and step count t >= 1.  theta, m1, m2: device float64 [n], updated in
 * place (m1 = m2 = 0 before the first step).  Asynchronous on `stream`. */
int afm_adam_step(double* theta, const float* grad, double* m1, double* m2, int64_t n, double lr,
                  double beta1, double beta2, double eps, int64_t t, void* stream);

/* ---- systems, neighbour lists, workspaces --------------------------------- */
typedef struct {
  int64_t n_atoms;
  int64_t n_struct;
  const double* pos;       /* [n_atoms, 3] */
  const int32_t* species;  /* [n_atoms] */
  const double* cell;      /* [n_struct, 3, 3] */
  const uint8_t* pbc;      /* [n_struct] */
  const int64_t* seg;      /* [n_struct + 1] atom offsets, seg[0] = 0 */
} afm_system;

/* CSR edge list in canonical order.  row_ptr[i]..row_ptr[i+1] are the edges
 * of central atom i; col = neighbour atom j; shift = image n (int8 x 3);
 * rev = index of (j, i, -n).  n_edges and status are single device words. */
typedef struct {
  int64_t capacity;        /* edges the col/shift/rev arrays can hold */
  int64_t* row_ptr;        /* [n_atoms + 1] */
  int32_t* col;            /* [capacity] */
  int8_t* shift;           /* [capacity, 3] */
  int32_t* rev;            /* [capacity] */
  int64_t* n_edges;        /* [1] */
  int32_t* status;         /* [1] AFM_FLAG_* bits, OR-ed, never cleared by the library */
} afm_nlist;

/* Device scratch memory for one (model, system size, edge capacity).
 * Filled by afm_workspace_plan; the caller allocates `bytes` bytes of device
 * memory (256-byte aligned) and stores the pointer in `ptr`.  Edges are
 * processed in chunks of whole rows of at most chunk_edges + max_row edges;
 * chunk_edges is chosen so the plan fits in max_bytes (0 = no limit).  A
 * row longer than max_row sets AFM_FLAG_CAPACITY.  With model == NULL the plan
 * holds only the scratch of afm_build_neighbors. */
typedef struct {
  void* ptr;
  int64_t bytes;
  int64_t n_atoms;
  int64_t n_struct;
  int64_t edge_capacity;
  int64_t chunk_edges;
  int64_t n_chunks;
  int64_t max_row;
  int32_t precision;
  int32_t with_second_order;  /* plan holds the double-backward state */
} afm_workspace;

int afm_workspace_plan(const afm_model* model, int64_t n_atoms, int64_t n_struct,
                       int64_t edge_capacity, int64_t max_bytes, int32_t with_second_order,
                       afm_workspace* ws /*host, out*/);

/* Abstract ("strictly-local") and Model Training (radial cutoff): build the
 * canonical edge list of every structure at cutoff r_list (>= the model
 * cutoff; the surplus is an MD skin).  The inclusion test is evaluated in
 * float64 exactly as d2 = (dx*dx + dy*dy) + dz*dz < r_list*r_list with
 * delta = (r_j - r_i) + ((n0*a + n1*b) + n2*c), no fused multiply-add.
 * Periodic structures enumerate every image with |n_k| <= ceil(r / w_k)
 * (w_k the perpendicular widths).  Uses the workspace's scratch area.  If
 * the edges do not fit, *n_edges holds the required count, AFM_FLAG_CAPACITY
 * is set and col/shift/rev are left unspecified. */
int afm_build_neighbors(const afm_system* sys, double r_list, afm_nlist* nl,
                        const afm_workspace* ws, void* stream);

/* Model Training: per-atom energies e_atom[n_atoms] (float64) and
 * per-structure energies e_struct[n_struct] (float64).  Leaves in `ws` the
 * state afm_backward_forces needs (the same sys/nl/ws must follow). */
int afm_forward_energy(const afm_model* model, const afm_system* sys, const afm_nlist* nl,
                       double* e_atom, double* e_struct, const afm_workspace* ws, void* stream);

/* Forces and virial as derivatives of the energy (they are the force and
 * stress terms of the training loss, Model Training): given the upstream
 * weights grad_e_struct[n_struct] (NULL = all ones) computes
 * forces[n_atoms,3] = -d(sum_s gE_s E_s)/dr and virial[n_struct,3,3]
 * (either may be NULL).  Accumulation in float64, deterministic (no atomics).
 * Must follow afm_forward_energy with the same arguments on the same stream. */
int afm_backward_forces(const afm_model* model, const afm_system* sys, const afm_nlist* nl,
                        const double* grad_e_struct, double* forces, double* virial,
                        const afm_workspace* ws, void* stream);

/* Energies, forces and virial in one pass (forward and adjoint per chunk). */
int afm_energy_forces(const afm_model* model, const afm_system* sys, const afm_nlist* nl,
                      double* e_atom, double* e_struct, double* forces, double* virial,
                      const afm_workspace* ws, void* stream);

/* ---- energies and forces without allocation -------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * what afm_energy_forces computes, with the same kernels, but its workspace
 * is a static device array inside the library (AFM_STATIC_SCRATCH_BYTES,
 * 256 MiB, on each GPU the library runs on, held until the process ends)
 * instead of a caller allocation.  The caller passes inputs and outputs as
 * for afm_energy_forces (nl built by afm_build_neighbors with any
 * workspace); the current device must be the model's.  No hipMalloc, no
 * allocating library call, no synchronisation.  The workspace is planned as
 * afm_workspace_plan would plan it with max_bytes = AFM_STATIC_SCRATCH_BYTES
 * (rows processed in chunks when the edges do not fit at once); a system
 * whose per-atom buffers and edge arrays alone exceed the array is rejected
 * with AFM_E_CAPACITY (e.g. ~15k atoms of the 2-layer, latent-256, c = 64,
 * l = 2 model fit; 1M atoms do not).  All calls on one GPU share its single
 * array: calls that overlap in time on one GPU (several streams or host
 * threads) race and must be serialised by the caller.  The array keeps the
 * last call's contents; every buffer this path reads is written first. */
#define AFM_STATIC_SCRATCH_BYTES (256LL << 20)
int afm_energy_forces_noalloc(const afm_model* model, const afm_system* sys, const afm_nlist* nl,
                              double* e_atom, double* e_struct, double* forces, double* virial,
                              void* stream);

/* Weight gradients for force and stress matching (Model Training: the loss
 * combines per-atom energy, force and stress errors): given upstream
 * grad_e_struct[n_struct], grad_forces[n_atoms,3] and
 * grad_virial[n_struct,3,3] (device, float64), writes
 *   grad_weights[n_params] = d/dtheta [sum_s gE_s E_s + sum_i gF_i . F_i
 *                                      + sum_s gW_s : W_s]
 * with W_s the virial of afm_backward_forces (device, float32, in the flat
 * weight layout, overwritten).  A NULL grad_e_struct, grad_forces or
 * grad_virial stands for zeros.  (A stress sigma_s = W_s / V_s enters as
 * gW_s = g_sigma_s / V_s.)  Needs a workspace planned
 * with with_second_order = 1.  FP32 models run its GEMMs on FP32 MFMA,
 * BF16 models on BF16 MFMA (operands rounded to bf16, FP32 accumulation);
 * the weight gradients accumulate in FP64 in a fixed order
 * (deterministic).  Built for per-path mixing at (l_max, layers, channels)
 * = (1, 1, 8), (2, 1, 8), (2, 2, 8 | 16 | 32 | 64 | 128) and (2, 3, 64);
 * other models (l_max = 3, dense mixing over two or more layers) get
 * AFM_E_UNSUPPORTED before anything is launched.  If grad_pos
 * (device, float64 [n_atoms, 3]) is not NULL it receives the position
 * gradient of the same objective, dJ/dr_i (overwritten; the cells are held
 * fixed): the reverse pass then also carries the adjoints of each edge's
 * basis (radial functions, envelope, spherical harmonics) and of their
 * tangents, differentiated per edge with respect to delta_e (second
 * derivatives of the basis) and scattered to the atoms like forces. */
int afm_backward_forces_backward(const afm_model* model, const afm_system* sys,
                                 const afm_nlist* nl, const double* grad_e_struct,
                                 const double* grad_forces, const double* grad_virial,
                                 float* grad_weights, double* grad_pos, const afm_workspace* ws,
                                 void* stream);

/* ---- edge-tile shape of the MLP chains --------------------------------------
 * The per-edge MLPs (two-body, latent and embedding; Methodology / Model
 * Training) run on BF16 MFMA in workgroup tiles of edges x wavefronts =
 * 64 x 8 (two workgroups per compute unit), 128 x 16 or 128 x 8 (one; the
 * last with twice the columns per wavefront).  Every edge's result is the
 * same with any shape (bit for bit); only the speed differs.  The shape is
 * a property of the model (default 64 x 8) and must not change between
 * afm_forward_energy and the afm_backward_forces that follows it.  Latent
 * widths above 256 are built for 64 x 8 only (AFM_E_UNSUPPORTED otherwise;
 * the tuner skips the other shapes and reports -1 for them).  For FP32
 * models the shape has no effect (afm_get_edge_tile reports 0 x 0). */
int afm_set_edge_tile(afm_model* model, int32_t edges, int32_t waves);
int afm_get_edge_tile(const afm_model* model, int32_t* edges /*host*/, int32_t* waves /*host*/);
/* Fused last layer: afm_energy_forces (and afm_md_step) run the last latent
 * layer's forward and its adjoint as one kernel, since the adjoint's seed
 * (sigma_Z escale w_eff) is known per edge before the layer runs; results are
 * bit for bit those of the separate kernels.  Built for BF16 models with the
 * 64 x 8 tile and latent widths up to 256; elsewhere, and with on = 0, the
 * separate kernels run.  Default on.  *active (may be NULL) reports whether
 * the model's current shape uses it. */
int afm_set_fused_last(afm_model* model, int32_t on, int32_t* active /*host*/);
/* Tuner: times afm_energy_forces on the caller's system, list and workspace
 * (1 warm-up + 3 timed evaluations per shape, HIP events on `stream`),
 * selects the fastest shape for the model and returns it in *edges, *waves
 * (0 for FP32 models).  With cache_path (host string, may be NULL) the
 * choice is looked up first in that JSON file, keyed on the device
 * architecture, the model's shape (w, c, l_max, layers, depth, two-body
 * widths, n_b, precision) and the mean number of edges per atom; a hit sets
 * the shape without timing (*from_cache = 1), a miss adds the measured
 * entry.  ms (host, 3 doubles, may be NULL) receives the mean evaluation
 * time of the shapes 64x8, 128x16 and 128x8.  Not for the hot path: it
 * synchronises the stream, allocates and frees scratch outputs, and
 * overwrites the workspace. */
int afm_tune_edge_tile(afm_model* model, const afm_system* sys, const afm_nlist* nl,
                       const afm_workspace* ws, const char* cache_path /*host or NULL*/,
                       int32_t* edges /*host*/, int32_t* waves /*host*/, double* ms /*host [3] or NULL*/,
                       int32_t* from_cache /*host or NULL*/, void* stream);

/* ---- molecular dynamics ---------------------------------------------------
 * Methodology (MD simulations, 0.5 fs time step): velocity Verlet in
 * float64 with a = F / m * 9.648533212e-3 A fs^-2 per (eV A^-1 amu^-1).  The
 * neighbour list (cutoff r_cut + skin) is rebuilt, after wrapping periodic
 * atoms by whole lattice shifts, before the force evaluation of every step
 * k with k % rebuild_every == 0 (k counts from state->step + 1).  Each step
 * writes (kinetic, potential) energies to energy_log[2 t], [2 t + 1]
 * (device, float64, n_steps pairs).  On entry state->forces must hold the
 * forces of the current positions (afm_energy_forces) and the list must be
 * current; state->step == 0 marks a fresh start (the positions become the
 * rebuild reference for the skin check).  An atom displaced by more than
 * skin/2 since the last rebuild sets AFM_FLAG_SKIN.  With use_graph != 0 and
 * a non-null stream, the n-step sequence is captured into a hipGraph on the
 * first call for a given phase (step % rebuild_every) and replayed after
 * that (the first call instantiates the graph: host-side setup).
 *
 * Canonical ensemble (the paper's NVT runs at 300 K, Results): with
 * t_target_K > 0 a single Nose-Hoover thermostat couples to all atoms, with
 * mass Q = g kB T tau_fs^2 (g = n_dof, or 3 n_atoms when n_dof <= 0),
 * integrated by the symmetric Trotter splitting (thermostat half step,
 * velocity Verlet step, thermostat half step; a half step advances xi by
 * dt/4 with G = (2 KE - g kB T)/Q, scales the velocities by
 * exp(-xi dt/2), advances eta by xi dt/2 and xi by dt/4 again).  The
 * thermostat state lives in `nh` (device, caller-owned, 4 doubles: xi
 * (fs^-1), eta, and two scratch words; zeros for a fresh start) so that
 * captured graphs carry it from replay to replay.  If thermostat_log is
 * non-null, each step writes Q xi^2/2 + g kB T eta (eV) to thermostat_log[t]
 * (KE + PE + this is conserved).  The energy_log KE is taken after the
 * thermostat scaling.  t_target_K > 0 needs tau_fs > 0 and nh != NULL
 * (else AFM_E_INVALID); t_target_K <= 0 is NVE and ignores the other
 * fields.  Changing t_target_K or tau_fs captures a new graph. */
typedef struct {
  double* pos;                   /* [n_atoms, 3] device, updated */
  double* vel;                   /* [n_atoms, 3] device, updated */
  double* forces;                /* [n_atoms, 3] device, updated */
  const double* mass_by_species; /* [n_species] device */
  double dt_fs;
  double skin;
  int32_t rebuild_every;
  int32_t use_graph;
  int64_t step;                  /* host, advanced by n_steps */
  double* energy_log;            /* [n_steps, 2] device */
  double* e_atom;                /* [n_atoms] device scratch */
  double* e_struct;              /* [n_struct] device scratch */
  double t_target_K;             /* NVT target temperature; <= 0: NVE */
  double tau_fs;                 /* NVT thermostat period */
  int64_t n_dof;                 /* NVT degrees of freedom; <= 0: 3 n_atoms */
  double* nh;                    /* [4] device: xi, eta, scratch (NVT) */
  double* thermostat_log;        /* [n_steps] device or NULL (NVT) */
} afm_md_state;

int afm_md_step(const afm_model* model, const afm_system* sys, afm_nlist* nl,
                afm_md_state* state, int32_t n_steps, const afm_workspace* ws, void* stream);

/* ---- tracing -------------------------------------------------------------
 * Per-stage HIP-event timers for profiling (host bookkeeping; do not enable
 * while capturing a graph).  afm_trace_enable(1) clears old records and
 * starts recording a start/stop event pair around every kernel stage of the
 * library on its stream; afm_trace_read waits for the recorded events and
 * returns, per stage name (e.g. "latent_fwd2"), the launch count and the
 * summed GPU time.  out: host, `max` entries; *n receives the stage count. */
typedef struct {
  char name[32];
  int32_t launches;
  double total_ms;
} afm_trace_stat;
int afm_trace_enable(int32_t enable);
int afm_trace_read(afm_trace_stat* out /*host*/, int32_t max, int32_t* n /*host*/);

/* Algorithmic work of each traced stage of afm_energy_forces for a model of
 * hyper-parameters `hp` (host; no device needed),
 * for roofline accounting (one entry per stage name that afm_trace_read
 * reports, e.g. "tp_bwd1").  Counts are what the mathematics needs, not what
 * the kernels issue: flops = 2 x multiply-adds of the stage's products (for
 * the MLP stages once per weight, although the BF16 path issues every
 * product as a hi + lo pair of MFMAs); bytes = compulsory HBM traffic, each
 * input read once and each output written once, in the BF16 path's storage
 * types (bf16 pre-activations, omega, s and dE/domega; float32 x, dE/dx,
 * dE/ds and geometry; per-atom tensors once per central atom).
 * kind: 0 = dense contraction (MFMA in the BF16 path), 1 = vector ALU /
 * memory stage, 2 = the dense-mixing GEMMs (mix_fwd / mix_bwd) on the
 * matrix cores: FP32 for FP32 models, bf16 operand pairs (three products
 * per block) for BF16 models.  out: host, `max` entries; *n receives the
 * stage count.  */
typedef struct {
  char name[32];
  int32_t kind;
  double flops_per_edge;
  double bytes_per_edge;
  double bytes_per_atom;
} afm_stage_cost;
int afm_stage_costs(const afm_hparams* hp /*host*/, afm_stage_cost* out /*host*/, int32_t max,
                    int32_t* n /*host*/);

/* Number of MD-step graphs afm_md_step currently keeps instantiated
 * (use_graph != 0).  A graph is keyed on the model's creation id and on
 * every pointer and scalar it was captured with; afm_model_destroy destroys
 * the graphs of that model, and the rest are destroyed at process exit. */
int64_t afm_md_graph_count(void);

/* ---- diagnostics ------------------------------------------------------- */
const char* afm_strerror(int code);
const char* afm_last_error(void);
/* Library version string. */
const char* afm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AFM_H_ */
