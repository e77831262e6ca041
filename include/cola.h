/*
 * cola.h -- C ABI of the MI355X (gfx950) COLA particle-mesh library.
 *
 * Method: Tassev, Zaldarriaga & Eisenstein, "Solving Large Scale Structure in Ten
 * Easy Steps with COLA" (arXiv:1301.0322).  The library evolves N = np^3 particles
 * with the COLA scheme: the time evolution of eq. (ALCtimestep), the frame
 * transforms of eq. (Lops) and the modified kick / drift operators of eq. (KDKALC),
 * with the force -(3/2) Om a d_x d_x^-2 delta of eq. (eom) computed by a
 * particle-mesh method (Section 2), and 2LPT initial conditions (Section 2,
 * Appendix A.3).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Particles: index p = (i*np + j)*np + k (k fastest), Lagrangian position
 *   q = (i, j, k) * box / np.  Per-particle vectors are SoA float arrays [3][np^3]
 *   (component d of particle p at d*np^3 + p), in Mpc/h.
 *   s  = x - q, the displacement (positions are stored as displacements);
 *   v  = v_res = T[s_res], the residual velocity of Appendix A.3 (scaled canonical
 *        velocity a^2 dx/dt / H0, in Mpc/h, measured by an LPT observer);
 *   s1, s2 = Zel'dovich and second-order displacements at a = 1 (D1(1) = 1,
 *        D2 ~ -3/7 D1^2).
 * - Mesh: nm^3 cells, C order [x][y][z], z fastest; value c is the cell centred at
 *   (c + 1/2) * box / nm.  Mass assignment is cloud-in-cell with particle mass
 *   (nm/np)^3, so the mean density is 1.
 * - Poisson solve: continuum kernel -1/k^2, spectral gradient i k, k = 0 and every
 *   mode with a Nyquist index set to zero.
 * - Every pointer argument named as device memory must be a device allocation of
 *   the current HIP device (e.g. a torch CUDA/HIP tensor).  Arrays are not checked
 *   for size: the caller owns them and must pass at least the stated length.
 * - stream is a hipStream_t (passed as void*; NULL = the default stream).  Every
 *   call that takes a stream only enqueues work on it: it neither synchronises
 *   nor allocates device memory, except that the first such call on a plan uploads
 *   the plan's small tables (twiddles, spectrum table) to the current device.
 * - ws is the caller-owned device workspace of at least cola_workspace_bytes()
 *   bytes, 256-byte aligned.  Calls that share a workspace must be ordered on one
 *   stream.
 * - A plan is not thread-safe: calls on one plan must not overlap in time (they
 *   update its resident-step record and trace buffers).  Different plans may be
 *   used from different threads.  The library keeps a process-wide count per
 *   workspace address (a few bytes each, never freed) to tell whether a workspace
 *   still holds what a plan's previous call left there.
 * - Status: 0 on success, a negative COLA_ERR_* code otherwise; no exception or
 *   abort crosses this ABI.  cola_strerror() describes a code; after COLA_ERR_HIP,
 *   cola_last_hip_error() returns the hipError_t of the calling thread.
 */
#ifndef COLA_H
#define COLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COLA_OK 0
#define COLA_ERR_INVALID (-1)          /* null pointer or inconsistent parameter */
#define COLA_ERR_UNSUPPORTED_SIZE (-2) /* np or nm not in the supported size list */
#define COLA_ERR_RANGE (-3)            /* step index out of range */
#define COLA_ERR_HIP (-4)              /* a HIP runtime call failed */
#define COLA_ERR_DEVICE (-5)           /* plan used on a different device than its tables */
#define COLA_ERR_WORKSPACE (-6)        /* the call needs more scratch than the library's static array */

/* Variant flags (eq. KDKALC is the default). */
#define COLA_FLAG_KDK_STD 0x1u      /* standard COLA discretisation, eq. (KDKALCstd) */
#define COLA_FLAG_NO_LPT_FRAME 0x2u /* plain PM leapfrog, eq. (KDKStd): s1 = s2 = 0 in the operators */
#define COLA_FLAG_LOG_A_STEPS 0x4u  /* timesteps uniform in log a (Appendix A.2) instead of in a */
#define COLA_FLAG_U1_DRIFT 0x8u     /* eq. (KDKALC) with u = 1 in the drift and u = a^nLPT in the kick (the
                                       variant of the footnote on u(a), Appendix A.3.2); ignored with
                                       COLA_FLAG_KDK_STD or COLA_FLAG_NO_LPT_FRAME */

/* Run configuration (Section 2 and Appendix A.3).  Plain data, copied by
 * cola_plan_create. */
typedef struct {
  int32_t np;       /* particles per side; supported: 16 24 32 48 64 96 128 192 256 384 512 768 1024 */
  int32_t nm;       /* mesh cells per side; same list; nm must be a multiple of np */
  double box;       /* periodic box side L [Mpc/h], > 0 */
  double omega_m;   /* matter density today, > 0 */
  double omega_l;   /* cosmological constant today; curvature = 1 - omega_m - omega_l */
  double h;         /* H0 / (100 km/s/Mpc), sets the BBKS shape Gamma = omega_m h */
  double n_s;       /* primordial spectral index */
  double sigma8;    /* rms linear density in 8 Mpc/h top-hat spheres at a = 1, > 0 */
  double a_init;    /* initial scale factor (0.1 is z = 9), 0 < a_init < a_final */
  double a_final;   /* final scale factor (1 is z = 0) */
  int32_t n_steps;  /* number of COLA steps (10), >= 1 */
  double n_lpt;     /* u(a) = a^n_lpt of eq. (KDKALC) (-2.5), != 0 */
  uint32_t flags;   /* COLA_FLAG_* */
} cola_config;

typedef struct cola_plan_s *cola_plan;
typedef struct cola_ensemble_s *cola_ensemble;

/* Device particle arrays, each [3][np^3] floats (layout above), caller-owned. */
typedef struct {
  float *s;   /* displacement s = x - q */
  float *v;   /* residual velocity v_res */
  float *s1;  /* Zel'dovich displacement at a = 1 */
  float *s2;  /* second-order displacement at a = 1 */
} cola_particles;

/* Builds a plan: validates cfg and computes in FP64 on the host the growth factors
 * D1, D2, T[D1], T[D2], T^2[D1], T^2[D2] (Appendix A.1 and A.3), the kick and drift
 * factors of eq. (KDKALC) on the time grid of eq. (ALCtimestep), the BBKS spectrum
 * normalised to sigma8, and the FFT twiddles.  Host-only: needs no GPU.
 * *out receives the plan (NULL on failure). */
int cola_plan_create(const cola_config *cfg, cola_plan *out);

/* Frees the plan and the device tables it uploaded.  NULL is accepted. */
int cola_plan_destroy(cola_plan plan);

/* Bytes of workspace every call below needs: four nm^3 float meshes, the
 * per-step particle binning buffers (12 bytes per particle, three int arrays of
 * one entry per 8x8xtz tile, the halo faces of every tile) and two tile-sorted
 * copies of the particle state used by cola_run (104 bytes per particle). */
int cola_workspace_bytes(cola_plan plan, size_t *bytes);

/* Host copy of the per-step scalars (FP64).  out receives n = 13 * (n_steps + 1)
 * doubles: for i = 0..n_steps the row
 *   a_i, D1, D2, T[D1], T[D2], T^2[D1], T^2[D2] (all at a_i),
 *   alpha_i  merged kick factor at a_i (eq. KDKALC; half-kicks at i = 0 and i = n),
 *   beta_i   drift factor of step i (0 for i = n),
 *   dD1_i, dD2_i  D1(a_{i+1}) - D1(a_i), D2(a_{i+1}) - D2(a_i) (0 for i = n),
 *   a_{i+1/2} (0 for i = n), force factor (3/2) Om a_i.
 * len is the capacity of out in doubles.  Host-only. */
int cola_step_table(cola_plan plan, double *out, size_t len);

/* White noise: w[p] ~ N(0,1), p < np^3, from Philox4x32-10 (Salmon et al. 2011)
 * keyed by seed with counter = p / 4, Box-Muller on the four outputs.  w: device,
 * np^3 floats. */
int cola_noise(cola_plan plan, uint64_t seed, float *w, void *stream);

/* 2LPT initial conditions (Section 2; Appendix A.3): from white noise w (device,
 * np^3 floats, not modified) builds the linear field delta_k = w_k sqrt(P(k)/dp^3)
 * (dp = box/np, BBKS P at a = 1), writes s1 = -grad phi and s2 = grad phi2 with
 * lap phi = delta, lap phi2 = sum_{i<j} (phi_ii phi_jj - phi_ij^2), then the
 * initial state s = D1(a_init) s1 + D2(a_init) s2 and v = 0 (the 2LPT velocity
 * removed by L-(a_init), eq. Lops).  Writes all four arrays of p. */
int cola_init_2lpt(cola_plan plan, const float *w, const cola_particles *p, void *ws, void *stream);

/* Mean-1 CIC density of the particles at q + s: rho (device, nm^3 floats). */
int cola_density(cola_plan plan, const float *s, float *rho, void *ws, void *stream);

/* cola_density without a caller workspace and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  The particle binning buffers (8-byte key and rank plus a
 * 4-byte slot per particle, three int arrays of one entry per tile key, the scan sums
 * and the crowded-tile list) live in a file-scope device array of 256 MiB, one per GPU,
 * held from the first call on that GPU until the process ends: that covers every
 * configuration up to np = 256 (e.g. 256^3 particles on the 512^3 mesh).
 * s: device [3][np^3] displacements; rho: device nm^3 floats, the mean-1 CIC density
 * (identical to cola_density's).  Enqueues kernels on stream only: no hipMalloc, no
 * plan-table upload, no event creation.
 * Calls on one GPU share that GPU's array, so calls that overlap in time on one GPU
 * (different streams or threads) race and must be ordered by the caller; the array
 * keeps the last call's contents, which no call relies on (counters are cleared by
 * kernels every call).
 * Errors: COLA_ERR_INVALID for a null plan, s or rho, or a plan with tracing on;
 * COLA_ERR_WORKSPACE when the plan's binning buffers exceed 256 MiB (checked before
 * any device call); COLA_ERR_HIP if the array's device address cannot be obtained. */
int cola_density_noalloc(cola_plan plan, const float *s, float *rho, void *stream);

/* Density statistics of Section 3.1: the shell-averaged power spectra of the mean-1
 * CIC densities of two particle sets at q + s_a and q + s_b (device, [3][np^3]
 * floats each; s_b may be NULL for s_a alone), their cross spectrum, the
 * cross-correlation coefficient rho(k) = P_ab / sqrt(P_aa P_bb) (the square root as
 * in Appendix B) and n_max(k) = (2/3) rho / sqrt(1 - rho^2) of eq. (nmax).
 * out (device, 6 * (nm/2) doubles) receives rows r = 0..5 of nm/2 shells
 * s = round(|n|): mode count, P_aa, P_bb, P_ab, rho, n_max, with
 * P = <|delta_k|^2> L^3 / nm^6 over all modes of the full grid (modes with kz > 0
 * standing for their conjugates too).  Shell 0 (k = 0) is zero; shells are
 * complete for s < nm/2 (the kz = nm/2 plane is not formed).  With s_b NULL rows
 * 2..5 are zero.  The four workspace meshes are overwritten.  Errors:
 * COLA_ERR_INVALID for a null s_a or out. */
int cola_cross_power(cola_plan plan, const float *s_a, const float *s_b, double *out, void *ws, void *stream);

/* PM force of eq. (eom) at scale factor a: acc = -(3/2) Om a d d^-2 delta
 * interpolated to each particle (device, [3][np^3] floats). */
int cola_pm_force(cola_plan plan, const float *s, double a, float *acc, void *ws, void *stream);

/* One COLA step i (0 <= i < n_steps): the kick at a_i (merged half-kicks,
 * eq. KDKALC with a_c = a_i) using the PM force of the current s, then the drift
 * to a_{i+1} with a_c = a_{i+1/2}.  In: s(a_i), v(a_{i-1/2}) (v(a_0) for i = 0).
 * Out, in place: s(a_{i+1}), v(a_{i+1/2}).  With resident steps on
 * (cola_plan_set_resident_steps), a call that continues the previous resident call
 * starts from the state that call left in ws. */
int cola_step(cola_plan plan, int32_t i, const cola_particles *p, void *ws, void *stream);

/* Resident steps (off by default).  With on = 1, cola_step leaves in ws the updated
 * particle state sorted by mesh tile and its tile bins for the next step (as cola_run
 * does between its steps), and still writes s and v to the caller's arrays.  The next
 * cola_step (or cola_finish) of this plan continues from them, skipping the
 * re-binning and packing of the caller's arrays, when it is called with step index
 * i + 1 (n_steps for cola_finish), the same particle arrays and the same ws, and no
 * other call of this library has used ws in between; in every other case it starts
 * from the caller's arrays as with on = 0.  The caller must not change the particle
 * arrays (s, v, s1, s2) or ws between such calls: those changes would not be seen
 * (to change them, or to pass a new ws at the same address, call this function
 * again first: any call drops the record, so the next step starts from the arrays).
 * Results are identical bit for bit either way.  cola_run_checkpointed uses resident
 * steps internally regardless of this setting.  on = 0 or 1, else COLA_ERR_INVALID.
 * Host-only. */
int cola_plan_set_resident_steps(cola_plan plan, int32_t on);

/* Closing half-kick at a_n and L+(a_n) (eq. ALCtimestep, Lops).  p->v is updated
 * to v_res(a_n); x_out (device, [3][np^3]) receives the positions (q + s) mod box
 * and v_out (device, [3][np^3]) the full velocity v_res + T[D1] s1 + T[D2] s2. */
int cola_finish(cola_plan plan, const cola_particles *p, float *x_out, float *v_out, void *ws, void *stream);

/* Whole run: cola_init_2lpt, then the n_steps COLA steps and the closing kick of
 * cola_step / cola_finish.  Internally the particle state is kept in workspace
 * copies sorted by mesh tile between force evaluations, with the same arithmetic:
 * the results equal those of the step-by-step calls bit for bit (the mass deposit
 * sums 64-bit fixed point, independent of particle order).  On return p holds the
 * final s, v_res (in Lagrangian order) and the unchanged s1, s2. */
int cola_run(cola_plan plan, const float *w, const cola_particles *p, float *x_out, float *v_out, void *ws,
             void *stream);

/* Whole run as cola_run (Lagrangian-order steps), also storing the displacement
 * at every step for the adjoint: ckpt (device, [(n_steps + 1)][3][np^3] floats)
 * receives s(a_0), s(a_1), ..., s(a_n). */
int cola_run_checkpointed(cola_plan plan, const float *w, const cola_particles *p, float *x_out, float *v_out,
                          float *ckpt, void *ws, void *stream);

/* Bytes of workspace cola_run_adjoint needs (more than cola_workspace_bytes). */
int cola_adjoint_workspace_bytes(cola_plan plan, size_t *bytes);

/* Hand-written adjoint of the whole run.  Given the white noise w (device, np^3)
 * and the checkpoints ckpt of cola_run_checkpointed for that w, and the gradient
 * dL_drho (device, nm^3) of a loss L with respect to the final mean-1 CIC density
 * (cola_density of s(a_n)), writes dL_dw = dL/dw (device, np^3).
 * The reverse sweep applies, for i = n-1 .. 0, the transpose of the drift and kick
 * of eq. (KDKALC) with the force recomputed from s(a_i): the transpose of the PM
 * force is a CIC deposit of the cotangent, the conjugate k-space gradient and a
 * derivative-weighted CIC gather (CIC deposit and gather are each other's
 * transposes); then the transpose of the 2LPT initial conditions, where the
 * second-order source is quadratic in the Hessian of the linear potential.
 * The final half-kick does not move particles and does not enter.
 * Deterministic: the weighted deposits scale their weights by a power of two taken
 * from max |weight| (so that no cell sum can leave the range) and sum 64-bit fixed
 * point; a non-finite dL_drho or intermediate cotangent makes dL_dw NaN.
 * ws: at least cola_adjoint_workspace_bytes() bytes (not shared with a running
 * forward call). */
int cola_run_adjoint(cola_plan plan, const float *w, const float *ckpt, const float *dL_drho, float *dL_dw, void *ws,
                     void *stream);

/* Forward 3D real FFT on an n^3 grid, n = the plan's np or nm: out[kx][ky][kz]
 * (complex interleaved, kz = 0..n/2-1; the kz = n/2 plane is not produced) =
 * sum_x in[x] exp(-2 pi i k.x / n).  in, out: device, n^3 floats each (out holds
 * n * n * (n/2) complex); in is not modified; in == out is allowed. */
int cola_fft_r2c(cola_plan plan, int32_t n, const float *in, float *out, void *stream);

/* Inverse of cola_fft_r2c with the kz = n/2 plane taken as zero and the 1/n^3
 * factor applied (numpy irfftn of the padded half spectrum).  in is not modified
 * unless in == out. */
int cola_fft_c2r(cola_plan plan, int32_t n, const float *in, float *out, void *stream);

/* Tile shape of the strided FFT passes on the nm^3 mesh (a tuning knob; results
 * are identical for every valid shape).  pass 0 = the y passes, 1 = the x pass
 * with the Poisson multiplier; width = columns per tile, one of 4, 8, 16, or 0 for
 * the built-in default.  COLA_ERR_UNSUPPORTED_SIZE if the width does not divide
 * nm/2 or the tile's LDS exchange would exceed 144 KB.  Host-only. */
int cola_plan_set_fft_tile(cola_plan plan, int32_t pass, int32_t width);

/* Depth in cells (8, 16, 32 or 64) of the 8 x 8 x depth mesh tiles by which
 * particles are binned for the deposit and gather (a tuning knob; results are
 * identical for every depth: the mass deposit sums 64-bit fixed point and a
 * particle's arithmetic does not depend on its tile; the adjoint's weighted deposits
 * sum the same fixed point after an exact power-of-two scaling).  COLA_ERR_INVALID for other depths,
 * COLA_ERR_UNSUPPORTED_SIZE when depth does not divide nm.  Call
 * cola_workspace_bytes again afterwards.  Host-only. */
int cola_plan_set_bin_depth(cola_plan plan, int32_t depth);

/* Rotated planes for the nm^3 half spectrum between the y passes and the x pass of
 * the force, 2LPT and adjoint transforms (a tuning knob; results are identical bit
 * for bit either way, only the placement of rows in the workspace changes).  With
 * on = 1, row y of x-plane x is kept at row (y + r x) mod nm, r the x pass's inner
 * DFT length (32 for nm = 512 or 1024, 24 for 768).  The x pass reads one row of
 * every plane, and without rotation those rows are a power-of-two plane stride apart
 * (4 MB at nm = 1024), which concentrates them on few HBM channels.  on = 0 keeps
 * plain planes, on = -1 restores the built-in default (rotated for nm >= 1024);
 * other values give COLA_ERR_INVALID.  Transforms of length np (np != nm) use the
 * default for np.  cola_fft_r2c / cola_fft_c2r and the density statistics always
 * use plain planes.  Host-only. */
int cola_plan_set_fft_rotation(cola_plan plan, int32_t on);
/* The rotation in rows per plane that the plan uses for the nm mesh (0 = plain).
 * Host-only. */
int cola_plan_get_fft_rotation(cola_plan plan, int32_t *rows);

/* Current tuning: y-pass and x-pass tile widths (0 = built-in default) and bin
 * depth.  Host-only. */
int cola_plan_get_tuning(cola_plan plan, int32_t *y_width, int32_t *x_width, int32_t *bin_depth);

/* Autotuner: picks the FFT tile widths and the bin depth of the plan by timing one
 * PM force evaluation of the particles p (device) for every valid combination
 * (HIP events on stream, best of two repetitions) and keeps the fastest.  With
 * cache_path (a text file, may be NULL) a previous choice for the same
 * (np, nm, GPU architecture) is reused without measuring, and a new choice is
 * appended.  *used_cache (nullable) reports whether the cache answered.  ws holds
 * ws_bytes bytes (cola_tuning_workspace_bytes() lets every depth be tried; depths
 * whose binning buffers would not fit are skipped).  Call cola_workspace_bytes
 * again afterwards.  This call synchronises stream.
 * Results of the tuned plan equal the default's bit for bit: no tuning knob changes
 * the arithmetic (tile widths set how many columns a block transforms, the bin depth
 * which block adds a particle into fixed-point sums). */
int cola_autotune(cola_plan plan, const cola_particles *p, void *ws, size_t ws_bytes, void *stream,
                  const char *cache_path, int32_t *used_cache);
/* Workspace bytes that let cola_autotune try every tile depth. */
int cola_tuning_workspace_bytes(cola_plan plan, size_t *bytes);

/* Ensemble of independent realizations (possibly of different sizes), the
 * paper's intended use (Section 1: ensembles of mock catalogs).  Captures the
 * whole cola_run of every member k (plans[k], noise w[k], particles p[k], outputs
 * x_out[k], v_out[k], workspace ws[k]) once into a single hipGraph in which each
 * member is an independent branch, so small members run concurrently; members
 * must not share particles, outputs or workspaces.  Pointers are baked into the
 * graph: the buffers must stay allocated while the ensemble exists.  Plans must
 * have tracing off.  Creation uses private streams and does not run the graph. */
int cola_ensemble_create(int32_t n, const cola_plan *plans, const float *const *w, const cola_particles *p,
                         float *const *x_out, float *const *v_out, void *const *ws, cola_ensemble *out);
/* Runs every member once: a single graph launch on stream. */
int cola_ensemble_launch(cola_ensemble ens, void *stream);
/* One-shot batched run of an ensemble of realizations (Section 4: ensembles of
 * mock catalogues as the method's use): the members and buffers as in
 * cola_ensemble_create, captured into one graph, launched once on stream and freed.
 * Unlike the other calls that take a stream, it waits for that launch before it
 * returns (the graph must outlive it).  Each member's x_out, v_out and particles
 * equal those of cola_run bit for bit.  To run the same members again, create the
 * ensemble once and launch it. */
int cola_run_batched(int32_t n, const cola_plan *plans, const float *const *w, const cola_particles *p,
                     float *const *x_out, float *const *v_out, void *const *ws, void *stream);
/* Frees the graph (the caller synchronises any launch first).  NULL is accepted. */
int cola_ensemble_destroy(cola_ensemble ens);

/* Stage tracing (for profiling; off by default).  enable = 1: every kernel launch
 * of the calls above is bracketed by a pair of hipEvents recorded on the launch
 * stream.  enable = 2: only each COLA step of cola_run (deposit through the gather,
 * stage "run_step") is bracketed, so step times carry no per-kernel event cost.
 * enable = 0 turns tracing off; other values return COLA_ERR_INVALID.
 * cola_trace_read waits for the recorded events, fills ms[k] with the
 * summed elapsed milliseconds and launches[k] with the launch count of stage k
 * (k < cola_trace_stage_count(); n is the capacity of both arrays, which must be at
 * least that count) and clears the record.  Enabling or disabling clears it too.
 * Events are created on demand and reused; the calls above stay allocation-free
 * for device memory. */
int cola_trace_enable(cola_plan plan, int enable);
int cola_trace_read(cola_plan plan, double *ms, int32_t *launches, int32_t n);
int32_t cola_trace_stage_count(void);
/* Name of stage k (e.g. "fft_y_inv"), or NULL when k is out of range. */
const char *cola_trace_stage_name(int32_t stage);

const char *cola_strerror(int status);
int cola_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* COLA_H */
