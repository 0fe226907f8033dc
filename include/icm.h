/*
 * icm.h - C ABI of the MI355X (gfx950) incompressible Inertial Coupling
 * Method step.
 *
 * The library advances blob particles coupled to a fluctuating incompressible
 * fluid on a periodic staggered (MAC) grid by the second-order semi-implicit
 * step of Balboa Usabiaga, Delgado-Buscalioni, Griffith and Donev, "Inertial
 * coupling method for particles in an incompressible fluctuating fluid",
 * Sec. III.C (Summary of Algorithm, steps 1-9) with the inertial velocity
 * correction of App. C and the thermal drift of App. B.2. Every step of the
 * method runs in hand-written HIP kernels on the device; the host only
 * validates arguments, uploads/downloads state and enqueues work.
 *
 * Conventions shared by every entry point
 *  - Grid: Nx x Ny x Nz cells of side h (h = dx = dy = dz, Sec. III.A). Each
 *    N must be even, between 4 and 512, and have no prime factor other than 2
 *    and 3. A face field is three arrays (x, y, z components) of Nx*Ny*Nz
 *    values each, x fastest; v_x[k][j][i] sits at (i h, (j+1/2) h, (k+1/2) h),
 *    v_y at ((i+1/2) h, j h, (k+1/2) h), v_z at ((i+1/2) h, (j+1/2) h, k h).
 *  - Field values are double (ICM_FP64) or float (ICM_FP32_GRID); blob
 *    positions, velocities, masses and forces are always double, laid out as
 *    n_blobs x 3 (x,y,z interleaved). Positions are unwrapped: the library
 *    never folds them into the box, it wraps only when indexing the grid.
 *  - Host pointers are read or written only during the call. With
 *    ICM_PTRS_DEVICE the pointers must be device memory on the context's
 *    device; the copies are then enqueued on the context stream.
 *  - All device work is ordered on the stream given to icm_create. Calls that
 *    return data to host memory synchronise that stream first.
 *  - Every call returns an icm_status; on a negative status icm_last_error
 *    describes the problem. ICM_E_INVALID and ICM_E_UNSUPPORTED leave the
 *    context unchanged and usable. ICM_E_DEVICE and ICM_E_NUMERIC put it in an
 *    error state in which icm_step refuses to run until icm_set_state
 *    installs a new state.
 *  - One context must not be used from two host threads at once.
 */
#ifndef ICM_H
#define ICM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icm_ctx icm_ctx;

typedef enum {
    ICM_OK = 0,
    ICM_E_INVALID = -1,     /* bad argument or parameter                    */
    ICM_E_UNSUPPORTED = -2, /* valid request the library does not handle    */
    ICM_E_NOMEM = -3,       /* workspace too small or device allocation failed */
    ICM_E_DEVICE = -4,      /* a HIP call failed                            */
    ICM_E_STATE = -5,       /* context in error state / call out of order   */
    ICM_E_NUMERIC = -6      /* NaN/Inf or a blob moved more than h in a step */
} icm_status;

enum { ICM_FP64 = 0, ICM_FP32_GRID = 1 };

/* No-slip centring correction delta-u of step 4 (Sec. III.C):
 * NONE: delta-u = 0 (first order, most stable for very large dt);
 * VISCOUS: the lagged viscous term of Eq. (delta_u_nph_visc) (the paper's
 *          default for small Reynolds numbers);
 * FULL: Eq. (delta_u_nph), adding (J^{n+1/2} - J^n) v^n.                */
enum { ICM_SLIP_NONE = 0, ICM_SLIP_VISCOUS = 1, ICM_SLIP_FULL = 2 };

/* flags of icm_set_blobs / icm_set_state / icm_get_state */
enum {
    ICM_PTRS_DEVICE = 1u,   /* pointer arguments are device memory          */
    ICM_BLOBS_KICK = 2u,    /* icm_set_blobs: add to the fluid the impulse
                               v += P S(m~_f u) / rho that gives each blob the
                               velocity u at t = 0                           */
    ICM_STATE_PROJECT = 4u, /* icm_set_state: project the uploaded v onto
                               discretely divergence-free fields             */
    ICM_STATE_EQUILIBRIUM = 8u /* icm_set_state: replace v by a sample of the
                               discrete equilibrium N(0, kT/(rho h^3)) P drawn
                               from Philox block 3 of (seed, replica_id)     */
};

/* flags of icm_step */
enum {
    ICM_STEP_GRAPH = 1u     /* replay one recorded HIP graph of the whole step
                               (all replicas) per step instead of launching
                               its kernels one by one; the graph is recorded
                               on first use and again after icm_set_blobs.
                               Ignored while per-kernel timing is on.        */
};

/* Physical and numerical parameters of one replica (one periodic box). */
typedef struct {
    int32_t n[3];            /* Nx, Ny, Nz                                   */
    int32_t kernel;          /* 3 or 4: Peskin 3-point or 4-point kernel     */
    double h;                /* grid spacing (> 0)                           */
    double rho;              /* fluid density (> 0)                          */
    double eta;              /* shear viscosity (>= 0)                       */
    double kT;               /* temperature k_B T (>= 0; 0 = deterministic)  */
    double dt;               /* time step (> 0)                              */
    int32_t slip;            /* ICM_SLIP_*                                   */
    int32_t thermal_drift;   /* 1: spread the thermal drift of App. B.2 when
                                kT > 0; 0: omit it                           */
    uint64_t seed;           /* Philox key of the stochastic stress          */
    uint32_t replica_id;     /* Philox counter word distinguishing replicas  */
    uint32_t advection;      /* 1: add the advective term -D.(rho v v^T) to
                                step 2, lagged by Adams-Bashforth weights
                                3/2, -1/2 (Eq. (Adams_Bashforth)); fluxes in
                                the centred conservative form of the
                                staggered grid, which conserves momentum and,
                                for divergence-free v, energy (Sec. I.B).
                                A step with no previous term (the first, and
                                the first after icm_set_state or a kick)
                                uses the current term alone. Costs one more
                                face field of workspace. 0: off (default)  */
    double body_force[3];    /* uniform force density on the fluid           */
    double wca_eps;          /* WCA pair potential of Sec. IV.A (0 = off)    */
    double wca_sigma;        /* WCA diameter sigma of Eq. (WCA), the
                                parameter the paper's potential is written
                                in; the cutoff is 2^(1/6) sigma (a cutoff of
                                2h means sigma = 2h / 2^(1/6)) and must stay
                                below N h / 2 on every axis                  */
    double spring_k;         /* tether spring -k (q - c) per blob (0 = off)  */
    double spring_center[3];
    double kernel_shift;     /* s / h of the split (shifted) three-point
                                kernel of Sec. III.A.2, whose factor per axis
                                is the mean of phi3 shifted by -s/2 and +s/2:
                                a wider blob (larger hydrodynamic radius) on
                                the same grid. In (0, 1] with kernel 3 (the
                                support then spans four nodes); 0: the plain
                                kernel (default); other values, or a nonzero
                                shift with kernel 4: ICM_E_INVALID. The blob
                                volume dV = h^3 / <sum phi^2>^3 uses the
                                average of sum phi^2 over the blob position
                                within a cell, (1 + 2 A(s/h)) / 4 with A the
                                autocorrelation of phi3, since for the split
                                kernel that sum depends on the position     */
} icm_replica_params;

/* FP64 diagnostics of one replica, reduced on the device. */
typedef struct {
    double momentum[3];  /* rho h^3 sum v + sum m_e u: the total momentum that
                            the step conserves (Sec. II, after Eq. (no_slip);
                            App. C)                                          */
    double ke_fluid;     /* rho h^3 sum v^2 / 2                                 */
    double ke_blob;      /* sum m_e u^2 / 2                                     */
    double max_div;      /* max |D v| h / max |v| (0 for v = 0): the discrete
                            divergence the projection removes (Sec. III.D)   */
    double max_alpha;    /* advective CFL number alpha = V dt / h of
                            Eq. (alpha_beta), with V the largest magnitude of
                            any face velocity or blob velocity component     */
    int64_t step;        /* step counter n (feeds the Philox counter)          */
} icm_diag;

/* Bytes of device workspace icm_create needs for these replicas: the state
 * of the method at step n (the staggered face field v of Sec. III.A and the
 * blob positions, velocities and lagged slip terms of Sec. III.C), the
 * right-hand side and spectrum of the FFT solves of Sec. III.D, the
 * inertial-correction field of App. C, and per-blob stencil and cell-list
 * arrays. p: n_rep parameter blocks; max_blobs: n_rep capacities in
 * [0, 2^24). Writes *bytes; no device work.                                */
icm_status icm_workspace_bytes(int32_t n_rep, const icm_replica_params* p,
                               const int32_t* max_blobs, int32_t precision,
                               size_t* bytes);

/* Create a context of n_rep independent replicas (uneven grids allowed) that
 * are stepped together, each a periodic box of Sec. III.A advanced by the
 * step of Sec. III.C. precision: ICM_FP64 or ICM_FP32_GRID (blob state is
 * FP64 in both). workspace/bytes: device memory of at least
 * icm_workspace_bytes, owned by the caller and kept alive until
 * icm_destroy; NULL makes the library allocate (and free) it. stream: a
 * hipStream_t, or NULL for the null stream. On success *out receives the
 * context; the fluid starts at rest with no blobs.                          */
icm_status icm_create(int32_t n_rep, const icm_replica_params* p,
                      const int32_t* max_blobs, int32_t precision,
                      void* workspace, size_t bytes, void* stream,
                      icm_ctx** out);

/* Install n_blobs blobs in a replica (replacing any previous ones).
 * q: positions (required); u: velocities (NULL = 0); m_e: excess masses
 * (NULL = 0, each must exceed -m_f = -rho dV, Sec. I.A); f_const: constant
 * external forces (NULL = 0). Clears the lagged slip term.
 * Flags: ICM_PTRS_DEVICE, ICM_BLOBS_KICK.                                  */
icm_status icm_set_blobs(icm_ctx* ctx, int32_t replica, int32_t n_blobs,
                         const double* q, const double* u, const double* m_e,
                         const double* f_const, uint32_t flags);

/* Overwrite parts of a replica's state (checkpoint restore / test input):
 * the step-n quantities v^n, q^n, u^n and the lagged term
 * J^{n-1/2} L dv^{n-1/2} of Eq. (delta_u_nph_visc) that Sec. III.C step 4
 * reads.
 * v: face field in the context precision (NULL = keep); q, u, lag_c:
 * n_blobs x 3 blob arrays for the installed blobs (NULL = keep); step: the
 * step counter n that feeds the Philox counter (negative = keep).
 * Flags: ICM_PTRS_DEVICE, ICM_STATE_PROJECT, ICM_STATE_EQUILIBRIUM.
 * Clears the error state, and the advective history when v changes.        */
icm_status icm_set_state(icm_ctx* ctx, int32_t replica, const void* v,
                         const double* q, const double* u,
                         const double* lag_c, int64_t step, uint32_t flags);

/* Advance every replica by n_steps steps (Sec. III.C). Replicas of equal
 * grid shape, kernel and inertial path (all m_e = 0, or not) are advanced by
 * the same kernel launches. Work is enqueued on the context stream; the call
 * then synchronises once to check the numeric flag (NaN/Inf in a blob, or a
 * blob displacement above h in one step, which breaks the advective CFL
 * condition alpha < 1 of Sec. III.D) and returns ICM_E_NUMERIC if it was
 * raised. Flags: ICM_STEP_GRAPH (other bits: ICM_E_INVALID).               */
icm_status icm_step(icm_ctx* ctx, int64_t n_steps, uint32_t flags);

/* Launch shapes of the FFT passes and of the right-hand-side kernel for
 * one grid shape, as chosen by icm_autotune. FFT times are the five passes
 * of one spectral solve (x forward, y forward, z with the solve, y inverse,
 * x inverse) for all replicas of that shape, RHS times one launch of the
 * step-2 right-hand side (noise, viscous term, spread forces) followed by
 * those five passes, in microseconds.                                      */
typedef struct {
    int32_t n[3];          /* grid shape                                      */
    int32_t y_columns;     /* kx columns per workgroup of the y passes         */
    int32_t z_columns;     /* kx columns per workgroup of the z pass           */
    int32_t z_small_plan;  /* 1: fewer values per thread in the z pass (FP32)  */
    int32_t x_threads;     /* threads per workgroup of the x passes            */
    int32_t tuned;         /* 0: this shape takes the generic passes (nothing
                              to tune)                                        */
    int32_t rhs_z_chunk;   /* z planes per workgroup of the right-hand-side
                              kernel (4, 8 or 16; 0: chosen from the batch's
                              size)                                           */
    double us_default;     /* with the default shapes                         */
    double us_tuned;       /* with the chosen shapes                          */
    double us_rhs_default; /* RHS kernel and one solve's five passes, with the
                              size-based z chunk                              */
    double us_rhs_tuned;   /* the same with the chosen z chunk                */
} icm_tune_result;

/* Measure the launch-shape variants of the FFT passes and the z chunk of
 * the right-hand-side kernel on the context's own scratch buffers
 * (right-hand side, spectrum and inertial-correction fields, the spread's
 * z-chunk bins; the state v, q, u is not touched) and keep the fastest for
 * each grid shape. Enqueued on the context stream; synchronises. results: room for
 * `capacity` entries (may be NULL when capacity is 0); *n_results receives
 * the number of distinct grid shapes. A recorded step graph is dropped.     */
icm_status icm_autotune(icm_ctx* ctx, icm_tune_result* results, int32_t capacity, int32_t* n_results);

/* Install FFT launch shapes without measuring (for instance results saved
 * from an earlier icm_autotune): for each of the `count` entries, the
 * replicas whose grid shape equals n take y_columns and z_columns (1, 2, 4,
 * ..., 64), z_small_plan (0 or 1), x_threads (64, 128, 256 or 512) and
 * rhs_z_chunk (0, 4, 8 or 16); the time and `tuned` fields are ignored. Shapes only change how the passes are
 * launched, not their results beyond rounding. ICM_E_INVALID (context
 * unchanged) for a value outside those sets or a shape no replica has.
 * A recorded step graph is dropped.                                        */
icm_status icm_set_fft_shapes(icm_ctx* ctx, const icm_tune_result* shapes, int32_t count);

/* Read a replica's state at the current step n (v^n, q^n, u^n and the
 * lagged slip term of Sec. III.C) and its diagnostics. Any output may be
 * NULL. v: face field in the
 * context precision; q, u, lag_c: n_blobs x 3; diag: FP64 diagnostics.     */
icm_status icm_get_state(icm_ctx* ctx, int32_t replica, void* v, double* q,
                         double* u, double* lag_c, icm_diag* diag,
                         uint32_t flags);

/* Advective history of a replica with advection on: the advective term
 * D.(rho v v^T) of its last step (the lagged term of Eq. (Adams_Bashforth)),
 * in the context precision and laid out like v.
 * icm_get_advection_lag copies it to lag (NULL: skip) and sets *valid (NULL:
 * skip) to 1 if the next step will use it, 0 if the next step starts the
 * history with forward Euler. icm_set_advection_lag installs lag as that
 * term, so that the next step takes the Adams-Bashforth weights, or clears
 * the history when lag is NULL. With icm_get_state / icm_set_state (called
 * first: installing a field clears the history) this restores a run
 * exactly. ICM_E_INVALID if the replica has advection off.
 * Flags: ICM_PTRS_DEVICE.                                                  */
icm_status icm_get_advection_lag(icm_ctx* ctx, int32_t replica, void* lag, int32_t* valid, uint32_t flags);
icm_status icm_set_advection_lag(icm_ctx* ctx, int32_t replica, const void* lag, uint32_t flags);

/* Per-kernel timing of icm_step. With timing enabled, icm_step records a
 * pair of HIP events on the context stream around every kernel launch and
 * accumulates the elapsed time per phase (a fixed kernel family), so that a
 * kernel's average launch duration is ms[phase] / launches[phase]. Timing
 * adds a small host cost per launch; leave it off for throughput runs.     */
enum {
    ICM_PHASE_GATHER = 0,    /* J: interpolation of a face field at blobs    */
    ICM_PHASE_BLOB = 1,      /* per-blob FP64 updates (steps 1, 4, 8, 9)     */
    ICM_PHASE_FORCES = 2,    /* tether spring + WCA pair forces              */
    ICM_PHASE_RHS = 3,       /* step-2 right-hand side with Philox noise     */
    ICM_PHASE_SPREAD = 4,    /* S: spreading of forces / drift / momentum    */
    ICM_PHASE_FFT_X_FWD = 5, /* real-to-complex transform along x            */
    ICM_PHASE_FFT_Y_FWD = 6, /* complex transform along y                    */
    ICM_PHASE_FFT_Z_SOLVE = 7, /* z transform, Helmholtz + projection, inverse z */
    ICM_PHASE_FFT_Y_INV = 8, /* inverse transform along y                    */
    ICM_PHASE_FFT_X_INV = 9, /* complex-to-real transform along x            */
    ICM_PHASE_FIELD_OPS = 10, /* field clears and additions                  */
    ICM_PHASE_ADVECTION = 11, /* advective term of step 2 (advection on)     */
    ICM_NUM_PHASES = 12
};
typedef struct {
    double ms[16];         /* accumulated GPU time per phase (milliseconds) */
    int64_t launches[16];  /* number of timed launches per phase            */
} icm_timing;

icm_status icm_set_timing(icm_ctx* ctx, int32_t enable);
/* Copy the accumulated timing into *out; reset != 0 clears it afterwards.  */
icm_status icm_get_timing(icm_ctx* ctx, icm_timing* out, int32_t reset);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * spectral solve of icm_step and of icm_set_state(ICM_STATE_PROJECT) on
 * caller-owned fields, with no context and no allocation. It computes
 *   out = P (a + b lambda)^-1 rhs,
 * i.e. solves (a - b L) w + G pi = rhs, D w = 0 by Fourier diagonalisation
 * followed by projection (Sec. III.D), lambda = -L-hat >= 0 being the
 * symbol of minus the 7-point Laplacian; the k = 0 mode is divided by a and
 * not projected. a = rho/dt, b = eta/2 is step 2's Helmholtz operator, and
 * a = 1, b = 0 the projection of ICM_STATE_PROJECT.
 * n: Nx, Ny, Nz (even, 4..512, prime factors 2 and 3); h > 0; a > 0;
 * b >= 0. precision: ICM_FP64 (rhs, out are double) or ICM_FP32_GRID
 * (float). rhs, out: device face fields on the current device (3 arrays of
 * Nx*Ny*Nz values, x fastest, as v); out may equal rhs. stream: hipStream_t
 * of the current device (NULL: null stream). Work is enqueued only; the
 * call does not synchronise.
 * Every intermediate (spectrum, twiddle and symbol tables, descriptor) lives
 * in a 64 MiB device array that the library holds on each GPU it runs on
 * until the process ends: a grid whose spectrum needs more (above 128^3 in
 * FP64, about 4.5 M cells in FP32) is rejected with ICM_E_INVALID and a
 * message in icm_last_error(NULL), as are bad arguments. All calls on one
 * GPU share that array: calls that overlap on one GPU (two streams, two
 * host threads) race and must be serialised by the caller. Nothing in the
 * array needs to start at zero; each call rewrites what it reads.          */
icm_status icm_solve_noalloc(const int32_t n[3], double h, double a, double b, int32_t precision,
                             const void* rhs, void* out, void* stream);

/* Number of blobs currently installed in a replica (or -1 on a bad call). */
int32_t icm_num_blobs(const icm_ctx* ctx, int32_t replica);

/* Release the context and any memory the library allocated. NULL is a no-op. */
void icm_destroy(icm_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing
 * icm_create / icm_workspace_bytes when ctx is NULL). Never NULL.          */
const char* icm_last_error(const icm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ICM_H */
