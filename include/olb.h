/*
 * olb.h -- C-ABI of the MI355X (gfx950) D2Q25 off-lattice thermal Boltzmann
 * library: the per-stage update of the 25 distributions of the Gauss-Hermite
 * Q = 5 model of Busuioc, Ambrus, Biciusca and Sofonea (arXiv:1702.01690)
 * under third-order TVD Runge-Kutta.
 *
 * Conventions
 *   - Lattice nx * ny, node (x, y) at ((x + 1/2) ds, (y + 1/2) ds), 0-based.
 *   - Population index k = 5 * ky + kx; kx, ky = 0..4 index the ascending roots
 *     of He_5 (Table trots): p = (R[kx], R[ky]), R[2] = 0.
 *   - Host macroscopic arrays are double [ny][nx]; host distributions are
 *     double [25][ny][nx].
 *   - Units of Sec. 2.1 with m = k_B = 1.
 *
 * Ownership
 *   - The caller owns all host arrays; they are read or written synchronously
 *     inside the call and may be reused on return.
 *   - The caller owns device memory: olb_init receives a device workspace of at
 *     least olb_workspace_bytes() bytes (256-byte aligned) and a hipStream_t.
 *     The library never allocates device memory; the workspace and stream must
 *     outlive the context.  All device work is enqueued on that stream.
 *   - One context may be used by one host thread at a time.  Separate contexts
 *     are independent.
 *
 * Errors
 *   Every call returns an olb_status (0 = OLB_OK, negative = error).  No C++
 *   exception crosses this boundary.  After an error, olb_last_error() holds
 *   a human-readable message for that context.
 */
#ifndef OLB_H
#define OLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct olb_ctx olb_ctx;

typedef enum {
  OLB_OK = 0,
  OLB_E_ARG = -1,        /* null pointer, bad size, unsupported kind            */
  OLB_E_CFL = -2,        /* p_max dt / (m ds) >= 1 (CFL condition, Sec. 4.1)    */
  OLB_E_DOMAIN = -3,     /* n outside (0, 1/b), T <= 0, tau <= 0, T_w <= 0      */
  OLB_E_NONFINITE = -4,  /* a distribution became NaN or infinite during a step */
  OLB_E_WORKSPACE = -5,  /* workspace too small or misaligned                   */
  OLB_E_DEVICE = -6,     /* a HIP runtime call failed                           */
  OLB_E_STATE = -7       /* call out of order (e.g. step before set_fields)     */
} olb_status;

/* bc_y kinds: periodic; diffuse walls at both ends (Sec. 3.4.2); a specular
 * symmetry plane at the low end (Sec. 3.4.1: ghost rows mirror the interior
 * with p_y reversed) and a diffuse wall at the high end -- the half channel
 * of the planar-interface test (Sec. 5).
 * bc_x kinds: periodic, or OLB_BC_SPECULAR: specular planes at both ends of x
 * (Sec. 3.4.1 across x: halo columns mirror the interior with p_x reversed,
 * the carried n and Delta p mirror too; with walls in y, corner ghosts are
 * the mirror of the wall ghosts -- the box of the Laplace test, Sec. 6).
 * Needs nx >= 3.  All instances of a batch share bc_x and bc_y. */
enum { OLB_BC_PERIODIC = 0, OLB_BC_DIFFUSE = 1, OLB_BC_SPECULAR_DIFFUSE = 2, OLB_BC_SPECULAR = 3 };
enum { OLB_FP64 = 0, OLB_FP32_MIXED = 1 };

/* Problem statement of Secs. 2 and 3 of the paper:
 *   nx, ny      lattice nodes (frak N_1 x frak N_2); (ny + 6) * nx * 8 must
 *               stay below 2^31 (offsets within a distribution plane, with its
 *               6 ghost rows, are 32-bit byte offsets), else OLB_E_ARG: up to
 *               about 268 M nodes per instance, e.g. 16384 x 16377.
 *   ds, dt      lattice spacing and RK-3 time step (Eq. rk3).
 *   tau         BGK relaxation time (Eq. evolution), > 0.
 *   a, b        van der Waals EOS p^w = nT/(1 - bn) - a n^2 (Eq. vdw is
 *               a = 9/8, b = 1/3).
 *   sigma       surface-tension parameter of Eq. F_def, >= 0.
 *   bc_x, bc_y  per-axis boundary kind (the enum above).  Walls are
 *               supported across y only; the paper's walls across x map to
 *               this case by exchanging the axes.  Walls need ny >= 3.
 *   tw_lo/hi    wall temperature at y = -ds/2 / y = (ny - 1/2) ds.
 *   uw_lo/hi    tangential (x) wall velocity at the same walls.
 *   precision   OLB_FP64: FP64 storage and arithmetic throughout.
 *               OLB_FP32_MIXED: f stored in FP32 as f - w_k rho_ref; moment
 *               sums, the vdW pressure and the 49-point stencils in FP64; WENO,
 *               force term, collision and RK combine in FP32.
 *   rho_ref     reference density of the FP32 departure storage. */
typedef struct olb_params {
  int32_t nx, ny;
  double ds, dt, tau;
  double a, b, sigma;
  int32_t bc_x, bc_y;
  double tw_lo, tw_hi, uw_lo, uw_hi;
  int32_t precision;
  double rho_ref;
} olb_params;

/* Device workspace size for one context with these parameters. */
olb_status olb_workspace_bytes(const olb_params* p, size_t* bytes);

/* Validate p (CFL, tau > 0, sizes, kinds), carve the caller's workspace and
 * bind the stream (hipStream_t passed as void*; NULL = default stream). */
olb_status olb_init(const olb_params* p, void* dev_workspace, size_t bytes,
                    void* hip_stream, olb_ctx** out);

/* f <- f^eq(n, u, T) (Eqs. feq, g_alpha) from host fields [ny][nx]; checks
 * n in (0, 1/b), T > 0 and finiteness.  Synchronous. */
olb_status olb_set_fields(olb_ctx* c, const double* n, const double* ux,
                          const double* uy, const double* T);

/* Same from device double fields [4][ny][nx] (n, u_x, u_y, T planes), e.g.
 * restricted moments of a finer run.  The fields are checked on the device
 * first (OLB_E_DOMAIN leaves the previous state).  Synchronous. */
olb_status olb_set_fields_device(olb_ctx* c, const double* dev_fields);

/* Advance nsteps full RK-3 steps (Eq. rk3), each of three stages computing
 * L[f] of Eq. ecast: moments, EOS, 49-point force, force term of Eq. derf,
 * Hermite equilibrium, BGK, WENO-5 fluxes in x and y, wall ghosts
 * (Secs. 2.2-3.4).  Asynchronous on the context's stream: it only enqueues
 * kernels.  A non-finite density produced by a step sets a device flag that
 * the next synchronising call (olb_sync, olb_moments, olb_get_f) reports as
 * OLB_E_NONFINITE; f is left as computed. */
olb_status olb_step(olb_ctx* c, int32_t nsteps);

/* Wait for the context's stream; OLB_E_NONFINITE if any step since the last
 * olb_set_fields / olb_set_f produced a non-finite density. */
olb_status olb_sync(olb_ctx* c);

/* n, u_x, u_y, T of the current f into host arrays [ny][nx] (FP64), from the
 * moments of Sec. 2.2 (T = sum f |p - u|^2 / (2 n), D = 2).  Synchronises
 * the stream; reports OLB_E_NONFINITE like olb_sync (outputs are filled). */
olb_status olb_moments(olb_ctx* c, double* n, double* ux, double* uy, double* T);

/* Same moments into a caller-owned device buffer of 4 * nx * ny doubles
 * (n, then u_x, u_y, T planes).  Asynchronous. */
olb_status olb_moments_device(olb_ctx* c, double* dev_out);

/* Snapshot / restore of the full distribution, host double [25][ny][nx].
 * FP32_MIXED contexts convert on the fly.  Synchronous. */
olb_status olb_get_f(olb_ctx* c, double* f);
olb_status olb_set_f(olb_ctx* c, const double* f);

/* Wall densities n_w of the last stage (Eq. nw), host double [nx] each;
 * OLB_E_STATE without walls.  Synchronous. */
olb_status olb_wall_density(olb_ctx* c, double* nw_lo, double* nw_hi);

/* Block height of the stage kernel: 8 (default) or 16 waves per workgroup,
 * or 12 with FP32 storage (OLB_E_ARG otherwise); each workgroup updates
 * 63 x by nodes.  Results do not depend on it. */
olb_status olb_set_tile(olb_ctx* c, int32_t by);
/* FP32 departure storage keeps f - rho_ref b_kx b_ky, with the per-axis base
 * b = w (1 + h(0, T - 1)) of the equilibrium at rest and temperature T
 * (Eqs. feq, g_alpha; default T = 1, b = w).  A base near the state's
 * temperature keeps the stored departures small, so that their FP32
 * rounding stays small too.  T > 0 and finite (OLB_E_ARG otherwise); a set
 * distribution is re-based in place (the physical state is unchanged up to
 * FP32 rounding).  No effect on FP64 storage.  Synchronous. */
olb_status olb_set_base_temperature(olb_ctx* c, double T);
/* Order in which the stage launch visits the tiles: 0 = rows of the tile
 * grid (the reads of a tile row form long runs of consecutive addresses);
 * W > 0 = vertical strips W tiles wide, visited left to right, rows within a
 * strip (tiles that run together then share halos in L2: fewer bytes read).
 * Default: 0 with FP64 storage, 8 with FP32 storage, the faster of the two on
 * the 2048^2 FP64 and 4096^2 FP32 lattices.  Results do not depend on it
 * (bitwise).  OLB_E_ARG outside 0..1024. */
olb_status olb_set_tile_order(olb_ctx* c, int32_t strip);

/* Number of stage-kernel launches olb_step enqueues per RK-3 step (3), and
 * of wall-ghost launches (3 with walls, else 0). */
olb_status olb_launch_counts(const olb_ctx* c, int32_t* stage, int32_t* walls);

const char* olb_last_error(const olb_ctx* c);
const char* olb_strerror(olb_status s);
void olb_free(olb_ctx* c);

/* ------------------------------------------------------------------------
 * Batches: many independent instances advanced in lockstep, every RK stage
 * being ONE kernel launch over the tiles of all instances (plus one wall-
 * ghost launch with walls).  Instances may differ in every parameter except
 * precision and boundary kind.  Ownership, errors and host layouts are those
 * of the single-instance calls; i selects an instance (0 <= i < count).
 * ------------------------------------------------------------------------ */
typedef struct olb_batch olb_batch;

/* Workspace for count instances with parameters p[0..count-1]. */
olb_status olb_batch_workspace_bytes(const olb_params* p, int32_t count, size_t* bytes);
olb_status olb_batch_init(const olb_params* p, int32_t count, void* dev_workspace, size_t bytes,
                          void* hip_stream, olb_batch** out);
olb_status olb_batch_set_fields(olb_batch* b, int32_t i, const double* n, const double* ux,
                                const double* uy, const double* T);
olb_status olb_batch_set_fields_device(olb_batch* b, int32_t i, const double* dev_fields);
olb_status olb_batch_set_f(olb_batch* b, int32_t i, const double* f);
olb_status olb_batch_get_f(olb_batch* b, int32_t i, double* f);
/* nsteps RK-3 steps of every instance (all must have f).  Asynchronous. */
olb_status olb_batch_step(olb_batch* b, int32_t nsteps);
olb_status olb_batch_sync(olb_batch* b);
olb_status olb_batch_moments(olb_batch* b, int32_t i, double* n, double* ux, double* uy, double* T);
/* Moments of instance i into a device buffer of 4 * nx * ny doubles.  Async. */
olb_status olb_batch_moments_device(olb_batch* b, int32_t i, double* dev_out);
olb_status olb_batch_wall_density(olb_batch* b, int32_t i, double* nw_lo, double* nw_hi);
/* Replay olb_batch_step in HIP graphs of steps_per_graph RK-3 steps (rounded
 * up to even; 0 = direct launches).  Captured on first use; needs a
 * non-default stream.  Results are bitwise those of direct launches. */
olb_status olb_batch_use_graph(olb_batch* b, int32_t steps_per_graph);
olb_status olb_batch_set_tile(olb_batch* b, int32_t by);
/* olb_set_base_temperature for instance i of the batch. */
olb_status olb_batch_set_base_temperature(olb_batch* b, int32_t i, double T);
olb_status olb_batch_set_tile_order(olb_batch* b, int32_t strip);
/* Choose the launch configuration by timing trial_steps RK-3 steps of each
 * candidate on a uniform rest state of every instance, one parameter at a
 * time: the stage tile height (8, 16; also 12 with FP32 storage), then the
 * tile order (olb_batch_set_tile_order: rows, strips of 4, 8, 16), then,
 * when the batch replays HIP graphs (olb_batch_use_graph), the RK-3 steps
 * per graph (2, 10, 30).  None of them changes the results.  The choice is
 * read from / added to the JSON file cache_path (NULL: no cache), keyed by
 * precision, boundary kinds, instance count, total nodes and whether graphs
 * are used.  The trial overwrites the instances: set their fields
 * afterwards.  chosen_by (tile height) may be NULL. */
olb_status olb_batch_autotune(olb_batch* b, int32_t trial_steps, const char* cache_path,
                              int32_t* chosen_by);
/* The current launch configuration: tile height, tile order (strip width,
 * 0 = rows) and RK-3 steps per graph (0 = direct launches). */
olb_status olb_batch_launch_config(const olb_batch* b, int32_t* by, int32_t* strip, int32_t* steps_per_graph);
/* Tiles per stage launch and the current tile height. */
olb_status olb_batch_tiles(const olb_batch* b, int32_t* tiles, int32_t* by);
const char* olb_batch_last_error(const olb_batch* b);
void olb_batch_free(olb_batch* b);

/* ------------------------------------------------------------------------
 * Learned closure on a coarse lattice.  Neither the network nor its training
 * comes from the paper: it is an extension that corrects a 4x-coarser run of
 * the same method towards the restriction of a fine run.
 *
 * Network: moments (n, u_x, u_y, T) -> conv3x3(4->32) -> ReLU ->
 * conv3x3(32->32) -> ReLU -> conv3x3(32->4) -> correction (dn, du_x, du_y,
 * dT), periodic padding.  Inputs are normalised (m - in_mean) / in_scale,
 * outputs scaled by out_scale.  Convolutions run on the bf16 matrix cores
 * with FP32 accumulation; activations and back-propagated gradients are
 * rounded to bf16 (nearest even) between layers; parameters, gradients and
 * Adam moments are FP32.  Sums over nodes (gradients, loss, the projection's
 * channel sums) add per-workgroup partial sums in a fixed order, without
 * atomics: on one device and for one lattice size, every call with the same
 * inputs gives the same bits.
 *
 * Parameters: one FP32 vector of OLB_CLOSURE_NPARAM values
 *   [W1 (32x4x3x3) | b1 (32) | W2 (32x32x3x3) | b2 (32) | W3 (4x32x3x3) | b3 (4)]
 * with W[co][ci][ky][kx] weighting input (x + kx - 1, y + ky - 1).
 *
 * Moment planes are device double [4][ny][nx] (n, u_x, u_y, T), y outer.
 * A closure object holds no device memory of its own: the caller's
 * workspace (256-byte aligned, olb_closure_workspace_bytes) keeps
 * activations, parameters, gradients, Adam state and the per-workgroup
 * partial sums of the reductions over nodes.  Work is enqueued on
 * hip_stream; calls that return host values synchronise it.
 * ------------------------------------------------------------------------ */
#define OLB_CLOSURE_NPARAM 11588
typedef struct olb_closure olb_closure;

olb_status olb_closure_workspace_bytes(int32_t nx, int32_t ny, size_t* bytes);
olb_status olb_closure_init(int32_t nx, int32_t ny, void* dev_workspace, size_t bytes,
                            void* hip_stream, olb_closure** out);
/* Input normalisation and output scale, 4 values each (scales > 0). */
olb_status olb_closure_set_norm(olb_closure* c, const double in_mean[4], const double in_scale[4],
                                const double out_scale[4]);
/* Host FP32 parameters in / out; set_params also resets the Adam state.
 * Non-finite parameters: OLB_E_ARG. */
olb_status olb_closure_set_params(olb_closure* c, const float* params);
olb_status olb_closure_get_params(olb_closure* c, float* params);
/* Network output for device moments [4][ny][nx] -> device corrections
 * [4][ny][nx] (double), scaled by out_scale and projected as set by
 * olb_closure_set_conserve.  Asynchronous.  OLB_E_STATE before set_params. */
olb_status olb_closure_forward(olb_closure* c, const double* dev_moments, double* dev_delta);
/* The same through the training path's kernels (one launch per layer, the
 * activations in the workspace) instead of the fused one-tile-per-workgroup
 * kernel; without projection (mask 0) the two agree to the bit, with it to
 * FP64 rounding of the channel sums (which the two add in different
 * orders). */
olb_status olb_closure_forward_layers(olb_closure* c, const double* dev_moments, double* dev_delta);
/* Conservative projection of forward / apply: bit c of mask (c = 0 n,
 * 1 u_x, 2 u_y, 3 T) removes the lattice mean of that correction channel, so
 * that, e.g., the total mass is unchanged by apply (bit 0).  Default 7 (n,
 * u_x, u_y: the fine and coarse runs conserve mass and, to rounding and
 * stencil order, momentum; T keeps its mean because the fine run heats up
 * as its unresolved fluctuations decay).  The loss and gradients see the raw
 * network output.  OLB_E_ARG outside 0..15. */
olb_status olb_closure_set_conserve(olb_closure* c, int32_t mask);
/* Training pair: dev_moments (the coarse run's moments, the network input)
 * and dev_reference (the restricted fine moments at the same time), both
 * device [4][ny][nx].  Loss L = mean over nodes and the 4 channels of
 * (out - (reference - moments) / out_scale)^2 with out the normalised network
 * output; grad = dL/dparams (host FP32, OLB_CLOSURE_NPARAM values; loss may
 * be NULL).  Synchronous. */
olb_status olb_closure_gradients(olb_closure* c, const double* dev_moments, const double* dev_reference,
                                 float* grad, float* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * loss with learning rate lr.  loss may be NULL (then asynchronous). */
olb_status olb_closure_train_step(olb_closure* c, const double* dev_moments, const double* dev_reference,
                                  float lr, float* loss);
/* Correct a single-instance coarse lattice of the closure's size in place:
 * m = moments of f^n, dm = network(m), f <- f + f^eq(m + dm) - f^eq(m) at
 * every node where m + dm is admissible (finite, 0 < n < 1/b, T > 0); other
 * nodes are left as they are and counted in *skipped (may be NULL).  The
 * lattice's carried state is refreshed.  Synchronises both streams when the
 * lattice runs on another stream. */
olb_status olb_closure_apply(olb_closure* c, olb_ctx* coarse, int32_t* skipped);
/* Move the moments of a coarse lattice to dev_target [4][ny][nx] keeping its
 * non-equilibrium part: f <- f + f^eq(target) - f^eq(m) at nodes where the
 * target is admissible (others counted in *skipped).  The moments m before
 * the change go to dev_moments (device [4][ny][nx], may be NULL).  Used to
 * make training pairs along a coarse run held on the restricted fine one
 * (a perfect closure); needs no parameters.  Synchronisation as apply. */
olb_status olb_closure_nudge(olb_closure* c, olb_ctx* coarse, const double* dev_target, double* dev_moments,
                             int32_t* skipped);
const char* olb_closure_last_error(const olb_closure* c);
void olb_closure_free(olb_closure* c);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): olb_closure_forward without
 * a closure object or workspace.  Same kernels and bits (network output of
 * dev_moments, device double [4][ny][nx], scaled by out_scale and projected
 * by conserve_mask, into dev_delta, device double [4][ny][nx]); the
 * parameters come from dev_params, device FP32 [OLB_CLOSURE_NPARAM] in the
 * layout above, and the normalisation from the host arrays (as
 * olb_closure_set_norm).  The bf16 weight matrices and the projection's
 * partial channel sums live in a static device array of 40 KiB that the library
 * holds on every GPU it runs on until the process ends; the call allocates
 * nothing and enqueues three kernels on hip_stream (no memset).  Every call
 * on a GPU overwrites that array: calls that overlap on one GPU (other
 * streams, other threads) race.  nx, ny >= 1 with nx * ny < 2^30 and mask in
 * 0..15, else OLB_E_ARG; non-positive scales: OLB_E_ARG.  Asynchronous. */
olb_status olb_closure_forward_noalloc(int32_t nx, int32_t ny, const float* dev_params, const double in_mean[4],
                                       const double in_scale[4], const double out_scale[4], int32_t conserve_mask,
                                       const double* dev_moments, double* dev_delta, void* hip_stream);

/* Conservative restriction of fine moment planes [4][fny][fnx] to coarse
 * planes [4][fny/factor][fnx/factor]: n, n u and n (u^2 + 2T) (m = 1, D = 2)
 * are averaged over factor x factor blocks, then u and T recovered.  Both
 * device double; fnx, fny multiples of factor.  Asynchronous on hip_stream. */
olb_status olb_restrict(const double* dev_fine, int32_t fnx, int32_t fny, int32_t factor,
                        double* dev_coarse, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
