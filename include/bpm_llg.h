/*
 * bpm_llg.h -- C ABI of the MI355X batched finite-element LLG island solver and its learned
 * screen.
 *
 * The operation is the recording simulation of Kovacs et al., "Numerical optimization of
 * writer and media for bit patterned magnetic recording", J. Appl. Phys. 120, 013902 (2016):
 * the Landau-Lifshitz-Gilbert equation of an exchange-coupled composite island (Sec. II.B,
 * Fig. 3: soft layer on a hard layer, coupled through an interlayer exchange A_ex,int) driven by
 * a head field that moves down-track and rises in 0.1 ns plus a global field H_ext (Sec. II.A,
 * Sec. II.C).  The critical-field search of Sec. II.C (Fig. 4; Eqs. (1)-(2)) runs many such
 * simulations side by side; here they are instances of one batched launch.
 *
 * Conventions
 *   - SI units; fields are given as B = mu0 H in tesla.
 *   - Every call returns BPM_OK (0) or a negative status.  On failure bpm_last_error() gives a
 *     message owned by the context, valid until the next call on that context.
 *   - Host pointers are caller-owned and only read during the call (copied).  Device pointers
 *     (marked "device") must stay valid until the work queued on the given stream completes.
 *   - hip_stream arguments: the HIP stream the call's work is queued on; NULL selects the
 *     context's own non-blocking stream, which is not ordered with the legacy default stream --
 *     callers whose inputs come from other streams pass that stream (or synchronise first).
 *   - One context per host thread.  Calls on one context are not thread-safe.
 *   - A numerical failure of one instance (non-finite state, step underflow, step budget) does
 *     not fail the run: it is reported in bpm_result.status and the other instances continue.
 */
#ifndef BPM_LLG_H
#define BPM_LLG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BPM_OK = 0,
  BPM_EINVAL = -1,           /* bad argument (message says which) */
  BPM_ENOMEM = -2,           /* device or host allocation failed */
  BPM_EHIP = -3,             /* HIP runtime error */
  BPM_ESTATE = -4,           /* call out of order (e.g. results before a run) */
  BPM_ENONFINITE = -5,       /* per instance: magnetisation became non-finite */
  BPM_ESTEPUNDERFLOW = -6,   /* per instance: adaptive step fell below dt_min */
  BPM_EMAXSTEPS = -7         /* per instance: max_steps attempts used up */
};

enum { BPM_FIELD_UNIFORM = 0, BPM_FIELD_POLE = 1, BPM_FIELD_GRID = 2 };
enum { BPM_DP45 = 0, BPM_DP5_FIXED = 1, BPM_HEUN = 2 };

typedef struct bpm_ctx bpm_ctx;

/* Creates a context on HIP device `device`.  *out receives the handle.  tune_cache (nullable):
 * path of the launch-shape cache that bpm_autotune appends to and this call reads (NULL: the
 * environment variable BPM_TUNE_CACHE, if set; an empty string: no cache file). */
int bpm_create(bpm_ctx** out, int device, const char* tune_cache);
void bpm_destroy(bpm_ctx* ctx);
const char* bpm_last_error(const bpm_ctx* ctx);

/* ------------------------------------------------------------------------------------------ */
/* Mesh groups                                                                                */
/* ------------------------------------------------------------------------------------------ */
/* P1 tetrahedral island mesh.  The paper meshes the island with NETGEN (Sec. II.A); any
 * conforming mesh is accepted.  Layer 0 is the soft layer (on top, nearest the head), layer 1
 * the hard layer (Sec. II.B, Fig. 3).  The two layers are meshed separately: nodes on the
 * interface exist twice, once per layer, and iface lists the pairs (soft node, hard node).   */
typedef struct {
  int32_t n_nodes, n_tets, n_iface, pad_;
  const double* xyz;          /* host [3][n_nodes], metres (SoA) */
  const int32_t* tet;         /* host [n_tets][4]; orientation free */
  const int32_t* node_layer;  /* host [n_nodes], 0 soft / 1 hard */
  const int32_t* iface;       /* host [n_iface][2] (soft node, hard node), may be NULL if 0 */
} bpm_mesh;

/* Adds a mesh group: assembles the P1 exchange stiffness, charge operator, lumped volumes and
 * interface areas on the host and copies them to the device.  The dense magnetostatic operator
 * S (energy (mu0/2) b^T S b of the nodal charges b) is either copied from S_host ([n][n] FP64,
 * row-major) or, when S_host is NULL, assembled on the GPU from Gaussian charge blobs of
 * standard deviation demag_beta * V_tet^(1/3) at the tet centroids (demag_beta <= 0 selects the
 * default 0.29166..., the blob whose self-energy equals a uniformly charged ball).  The stored
 * operator is made exactly symmetric, S <- (S + S^T) / 2 (an energy operator is symmetric by
 * definition; the kernels read either triangle).
 * Errors: BPM_EINVAL for an empty or inconsistent mesh (bad indices, degenerate tets, a node
 * with no tet, an interface pair not of one soft and one hard node).                         */
int bpm_mesh_add(bpm_ctx* ctx, const bpm_mesh* mesh, const double* S_host, double demag_beta,
                 int32_t* mesh_id);

/* As bpm_mesh_add, choosing which device copies of S to keep (flags, any combination):
 *   BPM_KEEP_S64        row-major FP64 [n][ldS] (precision-64 runs);
 *   BPM_KEEP_S32        row-major FP32 [n][ldS] (precision-32 runs of every kind);
 *   BPM_KEEP_S32_TILES  FP32 upper triangle only, packed in 64 x 64 tiles: about half the bytes
 *                       of the row-major copy; read by the upper-triangle product of FP32 runs
 *                       with BPM_FLAG_SYMMETRIC_DEMAG and one workgroup per group (it is used for
 *                       them whenever kept).
 *   BPM_KEEP_S16_TILES  the same tiles stored in FP16: S times a power-of-two scale (which puts
 *                       the largest |S_kl| between 2^13 and 2^14) rounded to nearest, a quarter of
 *                       the row-major FP32 bytes; the product widens every entry to FP32 and
 *                       accumulates in FP32 (relative rounding of each entry <= 2^-11).  Used by
 *                       the same launches when the FP32 tiles are not kept.
 * A run needs a copy it can use (BPM_EINVAL otherwise): a group keeping only packed tiles runs
 * only in such launches (not in BPM_HEUN runs or cooperative launches); large batches of FP32
 * runs keep only the packed tiles. */
enum { BPM_KEEP_S64 = 1, BPM_KEEP_S32 = 2, BPM_KEEP_S32_TILES = 4, BPM_KEEP_S16_TILES = 8 };
int bpm_mesh_add_ex(bpm_ctx* ctx, const bpm_mesh* mesh, const double* S_host, double demag_beta,
                    int32_t flags, int32_t* mesh_id);

/* Copies the group's demag operator to host memory S_out [n][n] (FP64, or the widened FP32 copy
 * if only that is kept, or both triangles unpacked from the packed FP32 tiles, else from the
 * FP16 tiles divided by their scale). */
int bpm_mesh_get_S(bpm_ctx* ctx, int32_t mesh_id, double* S_out);

/* Copies the host-assembled quantities of a group: V [n], rowptr [n+1], col [nnz], K [nnz],
 * D [nnz][3] (D_{k,(j,a)} = integral phi_j d_a phi_k for row k, column j), aif [n]; each pointer
 * may be NULL.  *nnz receives the pattern size. */
int bpm_mesh_get_assembly(bpm_ctx* ctx, int32_t mesh_id, int32_t* nnz, double* V,
                          int32_t* rowptr, int32_t* col, double* K, double* D, double* aif);

/* ------------------------------------------------------------------------------------------ */
/* Instances                                                                                  */
/* ------------------------------------------------------------------------------------------ */
/* Per-layer material (index 0 soft, 1 hard): saturation magnetisation Ms (A/m), uniaxial
 * anisotropy K (J/m^3) along the unit axis, exchange stiffness A (J/m); interlayer exchange
 * A_int (J/m) across an interlayer of thickness delta_int (m), i.e. a surface coupling
 * A_int/delta_int (J/m^2) (Sec. II.B, Fig. 3); Gilbert damping alpha.                        */
typedef struct {
  double Ms[2], K[2], A[2], axis[2][3];
  double A_int, delta_int, alpha;
} bpm_material;

/* Applied field B(x, t) = B_peak r(t) f(x, t) dir + B_ext with the rise r(t) = min(t/t_rise, 1)
 * (Sec. II.A: the head field is scaled with a 0.1 ns rise; Sec. II.C: a global H_ext).
 *   BPM_FIELD_UNIFORM: f = 1.
 *   BPM_FIELD_POLE:    f = fx * fy, a synthetic pole moving with velocity v (Sec. II.A: the
 *     precomputed head field moves down-track over the bit):
 *       fx = (1 - tanh(sx / L_grad)) / 2,  sx = x - x_off[0] - v[0] t
 *       fy = (tanh((sy + W_pole/2)/L_grad) - tanh((sy - W_pole/2)/L_grad)) / 2,
 *            sy = y - x_off[1] - v[1] t.
 *   BPM_FIELD_GRID:    f = the trilinear interpolation, at s = x - x_off - v t, of a grid of field
 *     vectors (the paper samples the precomputed head field on a 2.5 nm grid and hands it to the
 *     recording simulation, Sec. II.A): grid is host [3][nz][ny][nx] FP32 in tesla (component,
 *     then z, y, x), node (i, j, k) at g_origin + g_h (i, j, k), nx, ny, nz >= 2, g_h > 0; f = 0
 *     outside the box the nodes span; dir is not used.  The grid is copied at
 *     bpm_instance_add (instances given equal grids share one device copy).
 * Positions x are mesh coordinates plus the instance offset.                                 */
typedef struct {
  int32_t kind, pad_;
  double B_peak, dir[3], t_rise, v[3], x_off[3], L_grad, W_pole, B_ext[3];
  const float* grid;          /* BPM_FIELD_GRID only (else may be NULL) */
  int32_t nx, ny, nz, pad2_;
  double g_origin[3], g_h;
} bpm_field;

/* Adds an instance on mesh group mesh_id.  offset (may be NULL = 0) translates the island;
 * m0 (host [3][n], may be NULL = +z everywhere) is normalised on upload; seed keys the thermal
 * noise of BPM_HEUN runs (Philox key = (low 32 bits, high 32 bits)).                          */
int bpm_instance_add(bpm_ctx* ctx, int32_t mesh_id, const bpm_material* mat,
                     const bpm_field* field, const double* offset, const double* m0,
                     uint64_t seed, int32_t* inst_id);

/* Couples instances (all on one mesh group) through far-field point dipoles at the island
 * centroids: B_J = mu0 sum_{I != J} (3 (mu_I . r^) r^ - mu_I) / (4 pi r^3), mu_I = sum_i Ms V_i
 * m_i, applied uniformly to island J.  Coupled instances share one clock (one adaptive step). */
int bpm_couple_dipoles(bpm_ctx* ctx, int32_t n, const int32_t* inst_ids);

/* Removes every instance (mesh groups stay). */
int bpm_clear_instances(bpm_ctx* ctx);

/* ------------------------------------------------------------------------------------------ */
/* Runs                                                                                       */
/* ------------------------------------------------------------------------------------------ */
/* precision: 32 or 64.  integrator: BPM_DP45 (Dormand-Prince 5(4), error-controlled with the
 * RMS norm of e / (atol + rtol max(|y_n|,|y_n+1|)), accept at <= 1, next step
 * dt clamp(0.9 err^-1/5, 0.2, 5), no growth right after a rejection, |m| restored after every
 * accepted step), BPM_DP5_FIXED (the same stages with dt_fixed, last step clipped to t_end),
 * BPM_HEUN (stochastic Heun with a Langevin field of variance 2 alpha kB T / (gamma Ms V_i dt)
 * per component, Philox4x32-10 noise keyed by the instance seed and counter (step, node)).
 * save_every: trajectory sample every k accepted steps (0 = first and last only); traj_cap:
 * samples kept per instance.  wg_per_group: workgroups cooperating on one mesh group (0 =
 * automatic, or the autotuned value).  flags: see below.                                                                                */
typedef struct {
  int32_t precision, integrator;
  double t_end, dt0, dt_fixed, rtol, atol, dt_min, temperature;
  int64_t max_steps;
  int32_t save_every, traj_cap;
  int32_t wg_per_group, flags;
} bpm_run_opts;

/* bpm_run_opts.flags: BPM_FLAG_SYMMETRIC_DEMAG lets FP32 runs of groups owned by one workgroup read
 * only the upper triangle of the symmetric demag operator (half the bytes of the dominant stream;
 * the order of the floating-point sums then varies from run to run).  Runs whose groups span
 * several workgroups keep each workgroup's rows of S in LDS for the whole launch when they fit
 * (the demag product then reads no S from HBM); BPM_FLAG_STREAM_S turns that off. */
enum { BPM_FLAG_SYMMETRIC_DEMAG = 1,
       BPM_FLAG_WG512 = 2,    /* 512-thread workgroups for the stepping kernel (default: 512 for
                                 runs of several mesh groups, else 256 unless tuned) */
       BPM_FLAG_STREAM_S = 4, /* stream S from global memory even where its rows fit in LDS */
       BPM_FLAG_WG256 = 8,    /* 256-thread workgroups whatever the default */
       BPM_FLAG_CONTINUE = 16, /* continue the previous DP5 run (see below) */
       BPM_FLAG_RELAX = 32     /* DP5 runs without the precession term: dm/dt = -gamma alpha /
                                  (1 + alpha^2) m x (m x B), a descent of the total energy (the
                                  relaxation step of the string method, bpm_string_reparam) */ };

/* BPM_FLAG_CONTINUE: instead of starting from m0 at t = 0, the run continues the last
 * BPM_DP45 / BPM_DP5_FIXED run of this context up to the new t_end (>= the previous end): the
 * magnetisation and first-stage slope of the last accepted step, the time, next step size and
 * growth cap of the controller, the step counters (max_steps counts from the first run), the
 * switching-time crossing state and the trajectory buffer carry over.  The instance set must not
 * have changed since that run (BPM_ESTATE otherwise); integrator and precision must match and
 * the launch shape and other flags of that run are kept; rtol, atol, dt_min, max_steps and
 * save_every are taken from this call.  A fixed-step run continues only with the same dt_fixed
 * and a previous end on its time grid (BPM_EINVAL).  The last step before each end is shortened
 * to land on it, so a run split at intermediate ends takes that step sequence; the adaptive
 * controller then resumes with the step it had planned before the shortening when that is longer.
 * Fixed-step runs split on their grid take the same steps as one run (the split step ends at the
 * requested end time, which can differ from the grid time by rounding). */

/* Queues a run of every instance on `hip_stream` (NULL = the context's own stream).  Asynchronous. */
int bpm_run(bpm_ctx* ctx, const bpm_run_opts* opts, void* hip_stream);
/* Waits for the run; returns the first ABI-level error of the run. */
int bpm_sync(bpm_ctx* ctx);

/* Autotuner of the launch shape: runs the current instances (one or many mesh groups) for
 * probe_attempts step attempts with each candidate number of workgroups per group
 * cand[0..n_cand) (a negative candidate -g means g workgroups of 512 threads instead of 256; for
 * batches of many islands, 1 = one 256-thread workgroup per island, two islands per compute unit,
 * and -1 = one 512-thread workgroup per island), times the stepping kernel with HIP events (per
 * attempt of the longest-running system) and keeps the fastest in *best.  ms_per_attempt (may be NULL)
 * receives the time per attempt of each candidate (INFINITY where a candidate cannot run).  The
 * choice is cached in the context (and appended to the tune_cache file of bpm_create) under (size bucket of N, instance count, precision), and
 * bpm_run uses it when wg_per_group is 0.  Results of the probe runs are discarded. */
int bpm_autotune(bpm_ctx* ctx, const bpm_run_opts* opts, int32_t n_cand, const int32_t* cand,
                 int64_t probe_attempts, int32_t* best, double* ms_per_attempt);

/* Per-instance result.  switched: hard-layer <m_z> < 0 at the end (writing succeeded, Sec.
 * II.C).  t_sw: first time the volume-averaged hard-layer m_z reaches 0 (linear interpolation
 * between accepted steps; NaN if it never does).  B_sw: |B_applied| at the island centroid at
 * t_sw.  energy: total energy (J) at t_reached.                                               */
typedef struct {
  int32_t status, switched;
  double t_sw, B_sw, mz_soft, mz_hard, t_reached, energy;
  int64_t n_accept, n_reject;
  double dt_min_used, dt_max_used, max_norm_dev;
} bpm_result;

int bpm_get_results(bpm_ctx* ctx, int32_t n, const int32_t* ids, bpm_result* out);
/* Trajectory samples [cap][9] = (t, <mx>, <my>, <mz> (moment weighted), <mz>_soft, <mz>_hard
 * (volume weighted), |B_app(centroid)|, dt, err). */
int bpm_get_trajectory(bpm_ctx* ctx, int32_t id, double* out, int64_t cap, int64_t* n_written);
/* Final magnetisation of an instance as FP64 [3][n] (the unit vectors of its nodes), into host
 * memory (dst_is_device = 0) or device memory (dst_is_device != 0; written by a kernel on the
 * context's stream, complete when the call returns). */
int bpm_get_m(bpm_ctx* ctx, int32_t id, void* dst, int32_t dst_is_device);
/* Wall time of the last run's kernels (ms, HIP events on the run stream) and launch data. */
int bpm_last_run_info(bpm_ctx* ctx, double* kernel_ms, int32_t* grid, int32_t* wg_per_group);
/* Launch layout of the last DP5 run (any pointer may be NULL): threads per workgroup, rows of S
 * kept in LDS per workgroup (0 = S streamed), CSR entries staged in LDS (0 = none), instances per
 * staged block of the demag right-hand sides, and dynamic LDS bytes per workgroup. */
int bpm_last_run_layout(bpm_ctx* ctx, int32_t* threads_per_wg, int32_t* s_rows_lds, int32_t* csr_cap_lds,
                        int32_t* rhs_block, int64_t* lds_bytes);


/* ------------------------------------------------------------------------------------------ */
/* Energy barrier: string method                                                              */
/* ------------------------------------------------------------------------------------------ */
/* The paper computes the energy barrier of the adjacent bit in the head's fringing field with a
 * minimum-energy-path method (nudged elastic band, Sec. II.C); here the simplified string
 * method runs on the same field and energy kernels.  A string is a chain of P images
 * m^0..m^{P-1} of one island (P instances on one mesh group, in chain order).  One iteration
 * relaxes every image by a BPM_FLAG_RELAX run and then calls bpm_string_reparam, which moves the
 * images back to equal spacing along the chain:
 *   d_k = || m^{k+1} - m^k ||_2 over all 3n node components, s_k = d_0 + ... + d_{k-1},
 *   image j goes to arc length j s_{P-1} / (P - 1), by linear interpolation between the two
 *   images whose arc lengths bracket it, and every node vector is normalised
 * (the end images stay where they are).  It reads the final magnetisation of the last
 * synchronised DP5 run, which must have run the current instance set (BPM_ESTATE otherwise),
 * computes on the GPU in FP64, and stores the new images as the instances' m0, so that the next
 * fresh run starts from them.  arclen (host, P values, may be NULL) receives s_0..s_{P-1} of the
 * images before the redistribution; the energies of those images are the bpm_result energies
 * of that run.  3 <= P <= 64.  Synchronous. */
int bpm_string_reparam(bpm_ctx* ctx, int32_t n_images, const int32_t* ids, double* arclen);

/* ------------------------------------------------------------------------------------------ */
/* Global optimiser: expected improvement of a kriging model                                  */
/* ------------------------------------------------------------------------------------------ */
/* The paper's optimiser (efficient global optimisation, Sec. II.A) models the objective on the
 * unit box as a constant mu plus a Gaussian process of variance sigma2 with correlation
 * R(a, b) = exp(-sum_l theta_l (a_l - b_l)^2), fitted to the n designs evaluated so far, and
 * evaluates next the design of largest expected improvement over the best value f_min.  With
 * R = L L' the training correlation matrix (any nugget included), alpha = R^-1 (y - 1 mu),
 * w = R^-1 1 and c = 1' w, the model at a candidate x with correlations r is
 *   yhat = mu + alpha' r,  s^2 = sigma2 (1 - r' R^-1 r + (1 - w' r)^2 / c),
 *   EI = (f_min - yhat) Phi(z) + s phi(z), z = (f_min - yhat) / s  (max(f_min - yhat, 0) if s = 0),
 * with r' R^-1 r = |L^-1 r|^2.  All pointers below are device memory, FP64:
 *   X [n][d] training points, theta [d], G [n + 2][n] = the rows of L^-1 (zeros above its
 *   diagonal), then alpha', then w'.
 * 1 <= d <= 16, n >= 1, c > 0, sigma2 >= 0.                                                    */
typedef struct {
  int32_t n, d;
  double mu, sigma2, c, f_min;
  const double* X;
  const double* theta;
  const double* G;
} bpm_gp;

/* EI (and, if non-NULL, yhat and s) at m candidates cand [m][d] in the unit box.  seed != 0:
 * the call first fills cand with uniforms from Philox4x32-10, key (seed low, seed high), counter
 * (index low, index high, l / 4, 0), word l mod 4, u = (w + 1/2) 2^-32 for coordinate l; seed = 0:
 * cand is read.  Work is queued on hip_stream (NULL = the context's stream).                   */
int bpm_gp_ei(bpm_ctx* ctx, const bpm_gp* gp, int64_t m, double* cand, uint64_t seed, double* yhat,
              double* s, double* ei, void* hip_stream);
/* Index of the largest of v [m] (device FP64, m >= 1), the lowest index among equal values, into
 * idx (device int64 [1]; -1 if every value is NaN, which never wins); queued on hip_stream (NULL =
 * the context's stream).  Uses a small stream-ordered temporary allocation. */
int bpm_argmax(bpm_ctx* ctx, const double* v, int64_t m, int64_t* idx, void* hip_stream);

/* ------------------------------------------------------------------------------------------ */
/* Learned screen                                                                             */
/* ------------------------------------------------------------------------------------------ */
/* The paper's optimizer proposes each new design from a Gaussian-process surrogate of the
 * objective and evaluates the one with the largest expected improvement (Sec. II.A).  Here a
 * multilayer perceptron 12 -> 256 -> 256 -> 256 -> 256 -> 3 (exact-erf GELU between layers),
 * trained on the solver's own results, scores whole rounds of candidates; the batched solver
 * re-verifies the best.  Outputs: z-scored switching field, z-scored log switching time, logit
 * of the switching probability.  Every operand of a matrix product is rounded to bfloat16 (round
 * to nearest even) and accumulated in FP32 on the matrix cores; bias, GELU, loss and Adam are
 * FP32.  Parameters are one flat FP32 vector: per layer W [out][in] row-major, then b [out].
 * X, Y, T, mask, score and idx arguments are DEVICE pointers; theta and grads are host pointers. */
typedef struct bpm_mlp bpm_mlp;

/* Number of parameters of the network (201475). */
int bpm_mlp_num_params(void);
/* Creates a network able to train on batches up to max_batch; theta (host, may be NULL = zeros). */
int bpm_mlp_create(bpm_ctx* ctx, int32_t max_batch, const float* theta, bpm_mlp** out);
void bpm_mlp_destroy(bpm_mlp* net);
/* Replaces the parameters (and resets the Adam moments and step count). */
int bpm_mlp_set_params(bpm_mlp* net, const float* theta);
int bpm_mlp_get_params(bpm_mlp* net, float* theta);
/* Y [n][3] = net(X [n][12]) with the fused inference kernel (activations stay on chip). */
int bpm_mlp_predict(bpm_mlp* net, const float* X, float* Y, int64_t n, void* hip_stream);
/* Loss L = (1/B) sum_b [ mask_b ((y0-t0)^2 + (y1-t1)^2) + softplus(y2) - t2 y2 ] and its gradient
 * (host outputs, either may be NULL), without changing the parameters.  T: [B][3], mask: [B]. */
int bpm_mlp_grads(bpm_mlp* net, const float* X, const float* T, const uint8_t* mask, int32_t batch,
                  float* loss, float* grads);
/* One Adam step (beta = 0.9, 0.999, eps = 1e-8) on the same loss; loss (host, may be NULL)
 * receives the loss before the step (this synchronises the stream). */
int bpm_mlp_train_step(bpm_mlp* net, const float* X, const float* T, const uint8_t* mask,
                       int32_t batch, float lr, float* loss, void* hip_stream);
/* n candidate designs, scaled features X [n][12] in [-1, 1]: X[i][f] = 2u - 1 (rounded to FP32), u = (w + 1/2) 2^-32,
 * w the words of Philox4x32-10 with key (seed low, seed high) and counter (i low, i high, f/4, 0). */
int bpm_sample_designs(bpm_ctx* ctx, uint64_t seed, int64_t n, float* X, void* hip_stream);
/* Indices of the k largest scores, ordered by (score descending, index ascending); NaN ranks
 * lowest.  0 < k <= min(n, 16384), n < 2^31.  idx: device int64 [k]. */
int bpm_topk(bpm_mlp* net, const float* score, int64_t n, int64_t k, int64_t* idx, void* hip_stream);
/* Allocation-free variant of bpm_topk, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same selection,
 * order and tie rule, with no hipMalloc, hipFree or other allocation.  Its scratch (histogram,
 * selection state, candidates, per-block tie counts) is one fixed area of 394496 bytes in device
 * memory per GPU, held by the library until the process ends; it is cleared by the call's own
 * kernels.  score: device [n]; idx: device int64 [k]; work is queued on hip_stream (NULL = the
 * context's stream).  Limits: 0 < k <= min(n, 16384), n <= 67108864 (BPM_EINVAL beyond).  Every
 * call on one GPU uses that GPU's one area: calls that overlap in time on the same GPU (other
 * streams, contexts or threads) race and must be serialised by the caller. */
int bpm_topk_noalloc(bpm_ctx* ctx, const float* score, int64_t n, int64_t k, int64_t* idx, void* hip_stream);
/* One screening round: sample n designs uniformly in the box [lo, hi] (host [12], finite lo < hi;
 * the uniforms u as bpm_sample_designs, x = lo + (hi - lo) u), write their network inputs to X
 * (log coordinates 2 log(x/lo) / log(hi/lo) - 1 where lo > 0, else 2u - 1), predict, score =
 * predicted switching logit where the thermal-stability proxy (K_s V_s + K_h V_h) / (kB 300 K) is
 * at least min_stability (else -inf), keep the top k.  The feature order is d, t_soft, t_hard,
 * Ms_soft, Ms_hard, K_soft, K_hard, A_int, psi, B_peak, alpha, t_rise.  X [n][12], Y [n][3],
 * score [n], idx [k] on device.  Errors: BPM_EINVAL for a bad size or range. */
int bpm_screen(bpm_mlp* net, uint64_t seed, int64_t n, int64_t k, const double* lo, const double* hi,
               double min_stability, float* X, float* Y, float* score, int64_t* idx, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* BPM_LLG_H */
