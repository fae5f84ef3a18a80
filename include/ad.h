/*
 * ad.h -- C ABI of the MI355X (gfx950) library for the all-pairs hydrodynamic
 * step of active spring dumbbell suspensions.
 *
 * Model (Putz, Dunkel, Yeomans, "CUDA simulations of active dumbbell
 * suspensions"):
 *   dX_i/dt = u_i = F_i/(6 pi eta a)
 *                 + 1/(8 pi eta) sum_{j != i} [F_j/r + r (r.F_j)/r^3],
 *   r = X_i - X_j                       (Sec. II, Eq. e:langevin at zero
 *                                        temperature; Eq. e:Mazur, Oseen part)
 *   (AD_RPY adds the finite-size correction of Eq. e:Mazur, second line)
 *   F = -grad U, U = sum_s k/2 (d_s - L_s(t))^2,
 *   L_s(t) = ell + lambda sin(omega t + phi_s), omega = 2 pi / T
 *                                       (Sec. II, Eq. e:swimmer_potential)
 * Dumbbell s owns spheres 2s and 2s+1. Positions advance with classical RK4
 * (default) or the paper's Heun predictor-corrector (Sec. V).
 *
 * Conventions shared by every entry point:
 *   - Every call returns an int status: AD_OK (0) or a negative AD_E* code.
 *     Nothing throws across the ABI. ad_last_error() gives the message of the
 *     last failure on that context.
 *   - Array pointers marked "device" are caller-owned device allocations;
 *     pointers marked "host" are caller-owned host memory. The library never
 *     frees caller memory and keeps no pointer to it after the call returns,
 *     except the workspace bound with ad_bind_workspace.
 *   - Positions, forces and velocities are row-major [N_total][3] float64
 *     (a contiguous (N, 3) tensor). Systems of an ensemble are concatenated
 *     in order; system b holds spheres [2*sum_{c<b} S_c, 2*sum_{c<=b} S_c).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return without waiting, unless stated.
 *   - The context owns host-side objects only; all device memory it uses
 *     lives in the caller's workspace.
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef AD_H
#define AD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define AD_OK 0
#define AD_EINVAL (-1)     /* bad argument: null pointer, size, parameter */
#define AD_ENOMEM (-2)     /* workspace too small or host allocation failed */
#define AD_EDEVICE (-3)    /* HIP runtime error */
#define AD_ESTATE (-4)     /* call out of order (no workspace or no state) */
#define AD_ENONFINITE (-5) /* non-finite velocity or coincident spheres */
#define AD_ERANGE (-6)     /* AD_FP32C steric path: more than 16 spheres within 1.5 steric_r
                              of one sphere, or a sphere moved more than steric_r/4 in one
                              stage (the candidate lists would be incomplete) */

/* arithmetic of the pair sum (ad_params.precision) */
#define AD_FP64 0      /* FP64, ascending j, no FMA: bitwise equal to a plain
                          sequential FP64 evaluation of the sum */
#define AD_FP64_TILED 1 /* FP64 pair math, j split across work-groups */
#define AD_FP32C 2     /* FP32 pair math on hi/lo-split positions with
                          compensated (TwoSum) accumulation over j; self and
                          dumbbell-partner terms, state and RK4 in FP64 */
#define AD_FP64_DENSE 3 /* the paper's own GPU design (Sec. V): every stage
                          assembles each system's full 3Nb x 3Nb pair tensor
                          (FP64, 72 Nb^2 bytes of workspace per system, at most
                          32 GiB in all) and multiplies it by the forces. An
                          HBM-bound baseline for comparison; same results as
                          AD_FP64 up to rounding order */

/* time integrator (ad_params.integrator) */
#define AD_RK4 0
#define AD_HEUN 1 /* Sec. V: x~ = x + dt u(x,t); x' = x + dt/2 (u(x,t) + u(x~,t+dt)).
                     With kT > 0 both stages add g xi, g = sqrt(2 kT dt/(6 pi eta a)):
                     the additive noise with constant C of Sec. V (Eq. e:cholesky on the
                     diagonal of H). xi: three standard normals per sphere and step, from
                     Philox4x32-10 (key = seed, counter = (sphere, step)) and Box-Muller. */

/* pair tensor (ad_params.tensor) */
#define AD_OSEEN 0 /* (I + rr/r^2)/(8 pi eta r), Sec. II, Eq. e:Mazur first line */
#define AD_RPY 1   /* Oseen plus the Rotne-Prager-Yamakawa-Mazur correction
                      2a^2/(24 pi eta r^3) (I - 3 rr/r^2), Eq. e:Mazur second line,
                      applied at every distance */

typedef struct ad_params {
    double a;        /* sphere radius, > 0 */
    double eta;      /* viscosity, > 0 */
    double k;        /* spring constant k_0 */
    double ell;      /* mean dumbbell length */
    double lambda;   /* stroke amplitude (0: passive dumbbells) */
    double T;        /* stroke period, > 0 */
    double dt;       /* time step, > 0 */
    double steric_k; /* steric repulsion strength; 0 disables (not in the paper) */
    double steric_r; /* steric contact distance, force steric_k (steric_r - r) for r < steric_r */
    int32_t precision;  /* AD_FP64 | AD_FP64_TILED | AD_FP32C | AD_FP64_DENSE */
    int32_t integrator; /* AD_RK4 | AD_HEUN */
    int32_t tensor;     /* AD_OSEEN | AD_RPY */
    int32_t reserved;   /* must be 0 */
    double kT;          /* thermal energy k_B T >= 0; > 0 needs AD_HEUN (additive noise, below) */
    uint64_t seed;      /* key of the noise generator */
} ad_params;

/* Launch shape of the pair kernel. Zero fields mean "library default for
 * this size". A work-group of wg threads holds wg/64/wj waves on distinct
 * target spheres (ipl per lane) and wj waves that split every j-tile.
 * AD_FP64 with fused = 0 validates ipl, jchunk, wg and wj but its pair
 * kernel does not use them: a work-group of a producer and a consumer wave
 * per 1, 2 or 4 target spheres (about N_total / 1024), every source of the
 * system in ascending order. */
typedef struct ad_launch {
    int32_t ipl;      /* target spheres per lane: 1, 2 or 4 (FP64 modes: 1 or 2; dense: 1) */
    int32_t jchunk;   /* source spheres per work-group, >= 64 (AD_FP64: whole system;
                         AD_FP64_DENSE: tensor columns of 64..1024 spheres per product item) */
    int32_t wg;       /* work-group size: 64 or 256 (AD_FP64_DENSE: 256 tensor rows) */
    int32_t wj;       /* waves splitting each j-tile: 1, or 4 with wg = 256 (AD_FP32C) */
    int32_t posmode;  /* AD_FP32C positions: 1 = hi/lo float pair, 2 = single float */
    int32_t fused;    /* 1: each step stage is one kernel whose work-groups hold their
                         system's sources in LDS and also do the stage update, 16 target
                         spheres per work-group (AD_FP32C, no steric forces, at most 6784
                         spheres per system with single-float or 4544 with hi/lo positions;
                         ad_mobility_apply still uses the other fields);
                         2: the same with 64 target spheres per 4-wave work-group, one per
                         lane, for ensembles of small systems (at most 6824 single-float or
                         4548 hi/lo spheres per system);
                         3: 4, 8 or 16 target spheres per work-group (about N_total / 256)
                         whose waves stream their share of the sources through a small LDS
                         slot each (AD_FP32C, or AD_FP64_TILED in FP64 arithmetic with
                         v_rsq_f64 refined by one Newton step and FMAs; no steric forces, any
                         system size; sources are padded to a multiple of 1024);
                         4: resident: one work-group per system keeps the whole system on
                         the compute unit and runs every stage of a run of steps (up to the
                         next record point) in one launch (AD_FP64 and AD_FP64_TILED: the
                         sequential FP64 sum, systems of at most 128 spheres; AD_FP32C: at
                         most 256; no steric forces; for small systems and their ensembles);
                         0: pair kernel and epilogue as two kernels */
} ad_launch;

#define AD_POS_HILO 1
#define AD_POS_SINGLE 2

typedef struct ad_ctx ad_ctx;

/* Create a context for nsys independent systems, system b holding
 * S_per_sys[b] >= 1 dumbbells (host array). Validates the parameters
 * (a, eta, T, dt > 0; finite values; known enums). *out receives the
 * context. No device memory is allocated. */
int ad_create(const ad_params* p, int32_t nsys, const int32_t* S_per_sys, ad_ctx** out);

/* Destroy a context (host objects and captured graphs only). NULL is a no-op. */
int ad_destroy(ad_ctx* ctx);

/* Bytes of device workspace the context needs with its current launch shape. */
int ad_workspace_size(const ad_ctx* ctx, uint64_t* bytes);

/* Bind a caller-owned device buffer of at least ad_workspace_size() bytes,
 * 256-byte aligned. The caller keeps it alive until ad_destroy or the next
 * bind. Rebinding drops the state (call ad_set_state again). */
int ad_bind_workspace(ad_ctx* ctx, void* dev_ptr, uint64_t bytes);

/* Choose the pair-kernel launch shape (autotuning). Fails with AD_ENOMEM if
 * the bound workspace is too small for it; the state is kept. */
int ad_set_launch(ad_ctx* ctx, const ad_launch* launch);
int ad_get_launch(const ad_ctx* ctx, ad_launch* launch);

/* Load a state: X (device, [N_total][3] f64), phases phi (device, [S_total]
 * f64), and the clock: step n starts at time t0 + n*dt, the state is at step
 * step0. The phases are copied to the host once, where (sin phi, cos phi)
 * are taken with libm (Eq. e:swimmer_potential by the addition theorem).
 * Clears the non-finite flag. Synchronises the stream. */
int ad_set_state(ad_ctx* ctx, const double* X, const double* phi, double t0, int64_t step0,
                 void* stream);

/* Checkpoint: copy the positions to X (device, [N_total][3] f64) and return
 * the clock (t0, current step) on the host. Synchronises the stream. */
int ad_get_state(ad_ctx* ctx, double* X, double* t0, int64_t* step, void* stream);

/* F = -grad U at positions X (device [N_total][3]) and time t, plus steric
 * forces when enabled (Eq. e:swimmer_potential). Uses the phases of the
 * loaded state. F: device [N_total][3]. */
int ad_forces(ad_ctx* ctx, const double* X, double t, double* F, void* stream);

/* u = M(X) F for an arbitrary force F (Eq. e:Mazur, Oseen part, self term
 * included), per system. X, F, u: device [N_total][3]. Does not change the
 * loaded state. */
int ad_mobility_apply(ad_ctx* ctx, const double* X, const double* F, double* u, void* stream);

/* Advance the loaded state by nsteps >= 0 steps. Asynchronous. */
int ad_step(ad_ctx* ctx, int64_t nsteps, void* stream);

/* ad_step plus records: after every record_every-th step, the dumbbell
 * centres (X_2s + X_2s+1)/2 go to centres[r] (device [nrec][S_total][3]) and
 * each system's mean sphere position to com[r] (device [nrec][nsys][3]),
 * nrec = nsteps / record_every. Either pointer may be NULL. Synchronises the
 * stream at the end and returns AD_ENONFINITE if a non-finite velocity or a
 * coincident sphere pair was met since ad_set_state (AD_ERANGE for the
 * steric candidate conditions above). */
int ad_run(ad_ctx* ctx, int64_t nsteps, int32_t record_every, double* centres, double* com,
           void* stream);

/* Synchronise the stream and report the flags (AD_OK, AD_ENONFINITE or AD_ERANGE). */
int ad_check(ad_ctx* ctx, void* stream);

/* Capture runs of 16, 4 and 1 steps into HIP graphs (at the first
 * ad_step/ad_run after enabling, uploaded to the device on that call's
 * stream) and replay them, longest first, for ad_step/ad_run (enable != 0),
 * or launch kernels directly (enable == 0, the default). */
int ad_use_graph(ad_ctx* ctx, int32_t enable);

/* Measurement support. With enable != 0, ad_step/ad_run launch kernels
 * directly (no graph) and bracket every launch of the pair-sum kernel (with
 * launch.fused = 1, 2 or 3, the stage kernel, which also does the stage update; with
 * launch.fused = 4, each launch of the resident kernel; with
 * AD_FP64_DENSE, the assembly and product together) with HIP events on the
 * call's stream; ad_profile_read synchronises and returns the summed duration
 * (ms) and number of those launches since enabling. */
int ad_profile_pairs(ad_ctx* ctx, int32_t enable);
int ad_profile_read(ad_ctx* ctx, double* total_ms, int64_t* launches);

/* Measurement support: the issue rate of the FP32 pair term's instruction
 * mix with operands in registers (kind 0: single-float positions, 2: hi/lo
 * positions, 3: single-float into four independent accumulators) or of
 * independent FMA chains (kind 1), in `blocks` work-groups
 * of 256 threads, `iters` trips of 8 terms per thread. sink: device
 * [blocks*256] f32 (results, kept from being optimised away); clk: device [2]
 * i64, zeroed by the caller, receives the longest life of a work-group in
 * shader cycles (over the kernel's duration: the shader clock under the
 * load) and the sum over work-groups. Asynchronous on stream. */
int ad_valu_probe(int32_t kind, int32_t blocks, int32_t iters, float* sink, long long* clk, void* stream);

/* ---- Stroke-averaged far-field equations (Sec. III, Eqs. e:eom, J, K) ----
 * For S dumbbells with centres R, unit axes N and phases phi:
 *   dR_s/dt = sum_{r != s} J^{sr},  dN_s/dt = -(I - N_s N_s) sum_{r != s} K^{sr},
 * with J ~ |D|^-4 and K ~ |D|^-5 the stroke-averaged pair terms (uses a, ell,
 * lambda and T of p; the other fields are ignored). R, N, dR, dN: device
 * [S][3] f64; phi: device [S] f64. Context-free and asynchronous unless
 * stated. */

/* dR/dt and dN/dt at (R, N). */
int ad_sa_rhs(const ad_params* p, int32_t S, const double* R, const double* N, const double* phi,
              double* dR, double* dN, void* stream);

/* Bytes of device workspace ad_sa_run needs for S dumbbells. */
int ad_sa_workspace_size(int32_t S, uint64_t* bytes);

/* nsteps RK4 steps of size dt, in place on R and N; every axis is scaled back
 * to unit length after each step. workspace: device, 256-byte aligned, at
 * least ad_sa_workspace_size bytes. Synchronises the stream at the end;
 * returns AD_ENONFINITE if two centres coincided. */
int ad_sa_run(const ad_params* p, int32_t S, double* R, double* N, const double* phi, double dt,
              int64_t nsteps, void* workspace, uint64_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of ad_mobility_apply, u = M(X) F for ONE system of N spheres
 * (N even, dumbbell s = spheres 2s and 2s+1), with no context, no workspace
 * and no allocation of any kind. p supplies a, eta, precision (AD_FP64,
 * AD_FP64_TILED or AD_FP32C; the default launch shape of that precision) and
 * tensor; the other fields are ignored. X, F, u: device [N][3] f64,
 * caller-owned. Asynchronous on `stream`. The pack, partial sums and work
 * list live in a 16 MiB device array that the library holds on every device
 * until the process ends; sizes that need more are refused with AD_ENOMEM
 * (every N up to 131072 fits, except AD_FP64_TILED with AD_RPY: up to
 * 62948). Every call on one device uses that device's one array: calls that
 * overlap on a device (other streams, other threads) race and must be
 * serialised by the caller. Non-finite velocities are not reported.
 * Errors: AD_EINVAL (null pointer, odd or too small N, bad parameter),
 * AD_ENOMEM, AD_EDEVICE; message via ad_last_error(NULL). */
int ad_mobility_apply_static(const ad_params* p, int32_t N, const double* X, const double* F, double* u,
                             void* stream);

/* Message of the last failure on ctx (never NULL; "" if none). With ctx ==
 * NULL: the last failure of ad_create or ad_mobility_apply_static on the
 * calling thread. */
const char* ad_last_error(const ad_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* AD_H */
