/*
 * fslbm.h -- C ABI of the MI355X free-surface lattice Boltzmann (FSLBM) library.
 *
 * One call of fslbm_step advances B independent domains by whole FSLBM time
 * steps of Schwarzmeier & Ruede, "Comparison of refilling schemes in the
 * free-surface lattice Boltzmann method" (arXiv 2207.14496):
 *   (a) D3Q19 stream-collide (Sec. 2.1, collision/streaming equations, Guo
 *       forcing) with the anti-bounce-back free-surface condition at interface
 *       cells (Sec. 2.2, boundary-condition equation) and half-way bounce-back
 *       at walls (Sec. 2.1);
 *   (b) interface mass exchange and fill-level update (Sec. 2.2, mass and
 *       mass-flux equations; Sec. 3.2, mass-change equation);
 *   (c) curvature from Parker-Youngs fill-level normals and the Laplace gas
 *       pressure (Sec. 2.2, gas/volume/Laplace pressure equations);
 *   (d) cell conversion with one of the five refilling schemes EQ, EQ+NEQ,
 *       GEQ, EXT, AVG (Sec. 2.2 conversion rules; Sec. 3.1);
 *   (e) excess-mass redistribution (Sec. 2.2, excess-mass equation).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Cells: domain b in [0,B), cell n = (z*ny + y)*nx + x in [0,N), N = nx*ny*nz.
 *   Walls (no-slip, half-way bounce-back) lie half a cell outside the box on
 *   every axis that is not periodic.
 * - Canonical fields (what init accepts and read_fields returns), all in
 *   DEVICE memory, C-contiguous:
 *     flags  uint8   [B][N]      FSLBM_LIQUID / FSLBM_INTERFACE / FSLBM_GAS
 *     pdf    double  [B][19][N]  post-collision PDFs f*_i of the last step
 *                                 (unshifted; gas cells read back as 0)
 *     mass   double  [B][N]      interface-cell mass m (Sec. 2.2); 0 elsewhere
 *     phi    double  [B][N]      fill level (liquid 1, gas 0)
 *     rho    double  [B][N]      sum_i f*_i (fluid cells; 0 in gas)
 *     vel    double  [B][3][N]   sum_i c_i f*_i / rho - g/2 (fluid cells)
 *   D3Q19 order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0) (-1,-1,0)
 *   (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1)
 *   (0,1,-1) (0,-1,1); the opposite of i >= 1 is i+1 (odd i) or i-1 (even i).
 * - Memory: the caller owns every byte.  The library never allocates device
 *   memory; it carves the caller's workspace (fslbm_workspace_bytes) and keeps
 *   only a small host-side context.  (fslbm_init_static instead takes a static
 *   array that the library's code object holds on each device.)  Inputs are read, never retained (the
 *   adjoint target pointer is the one exception, see fslbm_adjoint_spec).
 * - Streams: all device work is enqueued on params.stream (a hipStream_t;
 *   NULL = the null stream).  fslbm_init, fslbm_read_fields and
 *   fslbm_diagnostics synchronise that stream before returning; fslbm_step
 *   does not.
 * - Errors: every call returns an fslbm_status.  After a failure the context
 *   is poisoned (every later call returns the same status) and
 *   fslbm_last_error() describes the first failure.  No C++ exception crosses
 *   this boundary.
 */
#ifndef FSLBM_H
#define FSLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSLBM_OK = 0,
    FSLBM_EINVAL = -1,     /* invalid argument or initial state */
    FSLBM_ENOMEM = -2,     /* workspace too small / host allocation failed */
    FSLBM_EDEVICE = -3,    /* a HIP runtime call failed */
    FSLBM_EUNSTABLE = -4,  /* non-finite values or |u| > c_s found by diagnostics */
    FSLBM_ESTATE = -5      /* context poisoned by an earlier error */
} fslbm_status;

/* Refilling schemes of newly created interface cells (Sec. 3.1). */
typedef enum {
    FSLBM_REFILL_EQ = 0,      /* f_eq of the mean neighbour rho, u            */
    FSLBM_REFILL_EQ_NEQ = 1,  /* EQ + non-equilibrium part of the neighbour   */
                              /* best aligned with the interface normal       */
    FSLBM_REFILL_GEQ = 2,     /* EQ + Grad's approximation of f_neq           */
    FSLBM_REFILL_EXT = 3,     /* 2nd-order extrapolation along that direction */
    FSLBM_REFILL_AVG = 4      /* mean of the neighbours' PDFs                 */
} fslbm_refill;

/* How PDFs are stored in HBM.  All modes store shifted populations
 * s (f_i - w_i); F64 computes in double, the others in float.  Mass, fill level,
 * excess mass and the conversion thresholds are double in every mode. */
typedef enum {
    FSLBM_F64 = 0,
    FSLBM_F32 = 1,
    FSLBM_F16 = 2,   /* s = 2^10 keeps |f - w| away from the fp16 subnormal range */
    FSLBM_BF16 = 3
} fslbm_storage;

typedef enum { FSLBM_SRT = 0, FSLBM_TRT = 1 } fslbm_collision;

enum { FSLBM_LIQUID = 1, FSLBM_INTERFACE = 2, FSLBM_GAS = 4 };

/* Field bits of fslbm_read_fields. */
enum {
    FSLBM_FIELD_FLAGS = 1u << 0,
    FSLBM_FIELD_PDF = 1u << 1,
    FSLBM_FIELD_MASS = 1u << 2,
    FSLBM_FIELD_PHI = 1u << 3,
    FSLBM_FIELD_RHO = 1u << 4,
    FSLBM_FIELD_VEL = 1u << 5,
    FSLBM_FIELD_BUBBLE_PRESSURE = 1u << 6   /* [B][N] f64, bubble_model = 1 only */
};

typedef struct fslbm_params {
    int32_t nx, ny, nz;     /* cells per domain, each >= 1                          */
    int32_t batch;          /* B >= 1 independent domains of the same size          */
    int32_t periodic[3];    /* per axis: 1 periodic, 0 walls at both ends          */
    int32_t collision;      /* fslbm_collision                                      */
    int32_t storage;        /* fslbm_storage                                        */
    int32_t refill;         /* fslbm_refill                                         */
    double omega;           /* relaxation rate, in (0, 2) (omega+ for TRT)          */
    double trt_lambda;      /* TRT magic parameter (3/16 puts walls half-way)       */
    double gravity[3];      /* acceleration g, lattice units                        */
    double sigma;           /* surface tension (0 disables curvature)               */
    double p_volume;        /* constant gas (volume) pressure p_V, e.g. 1/3         */
    double eps_phi;         /* conversion threshold, e.g. 1e-2                      */
    const double *omega_b;  /* optional HOST array [B]: per-domain omega, or NULL   */
    const double *gravity_b;/* optional HOST array [B][3]: per-domain g, or NULL    */
    void *stream;           /* hipStream_t for all work                             */
    double smagorinsky_cs;  /* Smagorinsky constant C_S of the turbulence model
                             * (Sec. 2.1, turbulence model), >= 0; 0 disables it.
                             * Per cell tau = (tau0 + sqrt(tau0^2 + 2 C_S^2 Qbar /
                             * (rho c_s^4))) / 2 with tau0 = 1/omega, Qbar =
                             * sqrt(2 Q:Q), Q_ab = sum_i c_ia c_ib (f_i - f_eq_i)
                             * of the post-streaming populations, dx = 1 (the
                             * solution of nu_t = c_s^2 (tau - tau0) = C_S^2 Qbar /
                             * (2 rho c_s^2 tau)).  With TRT it sets omega+ = 1/tau
                             * and omega- follows from trt_lambda.                 */
    int32_t free_slip;      /* walls (Sec. 2.1): 0 no-slip (half-way bounce-back),
                             * 1 free-slip (specular: a population that would
                             * enter a wall comes back with its wall-normal
                             * velocity components reversed, in the cell shifted
                             * by the other components; the mass exchange follows
                             * the same path)                                        */
    int32_t bubble_model;   /* volume pressure (Sec. 2.2, p_V(t) = p_V(0) V(0)/V(t)
                             * of an enclosed gas volume): 0 the one constant
                             * p_volume; 1 per bubble.  A bubble is a connected
                             * set of gas and interface cells (D3Q19 links); a
                             * cell holds the gas volume max(0, 1 - phi).  A set
                             * that reaches the top layer (z = nz-1) is the
                             * atmosphere at p_volume; every other bubble carries
                             * the amount p V, handed on at each step to the
                             * bubbles that hold its cells (shared by their gas
                             * volume), so p V is kept, merges add, splits share
                             * one pressure.  Every bubble starts at p_volume.
                             * A step's bubble kernels run after the next
                             * step's bulk kernel (which finishes its excess
                             * work), before that step's interface kernel; the
                             * call's last step finishes its own.
                             * fslbm_step_timed and the reverse mode reject it.  */
    int32_t diag_every;     /* stability check period K (Sec. 4: the solver is
                             * stable while |u| stays below c_s = 1/sqrt(3)):
                             * 0 off; K > 0: fslbm_step runs the diagnostics
                             * of fslbm_diagnostics after every step whose
                             * count since the state was loaded is a multiple
                             * of K (each check synchronises the stream) and
                             * returns FSLBM_EUNSTABLE at the first check that
                             * finds a non-finite value or a speed above c_s in
                             * some domain, without running the remaining steps
                             * and without poisoning the context
                             * (fslbm_last_error says where).  The checks do not
                             * change the steps' arithmetic.                    */
} fslbm_params;

typedef struct fslbm_ctx fslbm_ctx;

/* Per-domain diagnostics (fslbm_diagnostics). */
typedef struct fslbm_diag {
    double total_mass;      /* sum of liquid rho + interface m + reservoir (Sec. 3.2) */
    double reservoir;       /* excess mass that found no interface receiver       */
    double max_speed;       /* max |u| over fluid cells                           */
    int64_t n_liquid, n_interface, n_gas;
    int32_t finite;         /* 1 if every fluid PDF, m and phi is finite          */
    int32_t pad;
} fslbm_diag;

/* Bytes of device workspace fslbm_init needs for these parameters.
 * Returns FSLBM_EINVAL for invalid parameters. */
fslbm_status fslbm_workspace_bytes(const fslbm_params *params, size_t *bytes);

/*
 * Create a context on the caller's workspace and load the initial state.
 *   workspace  device buffer of at least fslbm_workspace_bytes, 256-byte aligned;
 *              owned by the caller, borrowed until fslbm_destroy.
 *   flags, phi canonical device arrays (required).
 *   pdf        canonical f* [B][19][N] (device), or NULL: then f* = f_eq(rho, u)
 *              (Sec. 2.1 equilibrium) from rho [B][N] and u [B][3][N] (device,
 *              required in that case).
 *   mass       interface mass [B][N] (device) or NULL: then m = phi * rho on
 *              interface cells, with rho the given density when pdf is NULL
 *              and sum_i f*_i otherwise (Sec. 2.2, mass definition).
 * Rejects (FSLBM_EINVAL) omega outside (0,2), non-positive sizes, unknown enums,
 * flags other than the three cell types, liquid phi != 1 or gas phi != 0, and a
 * liquid cell with a gas D3Q19 neighbour (an open interface layer, Sec. 2.2).
 * On success *out receives the context; on failure *out is NULL.
 */
fslbm_status fslbm_init(const fslbm_params *params, void *workspace, size_t bytes,
                        const uint8_t *flags, const double *phi, const double *rho,
                        const double *u, const double *pdf, const double *mass,
                        fslbm_ctx **out);

/*
 * Allocation-free variant of fslbm_init, for callers that cannot allocate
 * device memory (code running under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The context's workspace is the library's
 * own static device array of FSLBM_STATIC_WORKSPACE_BYTES (64 MiB), one per
 * device, held from the first use on a device until the process ends; the
 * call uses the array of the current device (params->stream must belong to
 * it).  Arguments and validation as fslbm_init, without workspace and bytes;
 * the call calls no hipMalloc or hipFree and allocates no device memory
 * (only the small host-side context).
 * Errors: FSLBM_ENOMEM (with the needed size in fslbm_last_error(NULL)) when
 * fslbm_workspace_bytes exceeds the array; FSLBM_ESTATE while another context
 * made by this call is alive on the device (one at a time: they would share
 * the array); FSLBM_EDEVICE without a current device.  The array keeps what
 * the last context left; the call clears whatever must start at zero.
 * fslbm_destroy of such a context waits for its stream, then frees the array
 * for the next call.  Calls on the context from several host threads at once
 * race, as on any context.
 */
#define FSLBM_STATIC_WORKSPACE_BYTES 67108864u
fslbm_status fslbm_init_static(const fslbm_params *params, const uint8_t *flags, const double *phi,
                               const double *rho, const double *u, const double *pdf,
                               const double *mass, fslbm_ctx **out);

/* Enqueue nsteps >= 0 FSLBM time steps (a)-(e) on the context's stream.
 * Asynchronous: device-side failures surface at the next synchronising call.
 * Without surface tension, the excess-mass redistribution of each step but
 * the last runs inside the next step's bulk kernel; the state after the call
 * is the same. */
fslbm_status fslbm_step(fslbm_ctx *ctx, int32_t nsteps);

/* Run nsteps >= 1 full time steps (a)-(e) with direct kernel launches on the
 * context's stream; the bulk stream-collide kernel of every step (which, as in
 * fslbm_step, also runs the last step's excess-mass redistribution where that
 * is fused) is launched with start and stop HIP events stamped by its own
 * dispatch (hipExtLaunchKernelGGL), so each duration is the kernel's alone.
 * Synchronises,
 * then returns (HOST doubles, milliseconds) the summed duration of the bulk
 * kernels and the wall time of the whole sequence.  The state advances
 * exactly as fslbm_step. */
fslbm_status fslbm_step_timed(fslbm_ctx *ctx, int32_t nsteps, double *bulk_ms, double *total_ms);

/* Select the refilling scheme (fslbm_refill) used by subsequent steps. */
fslbm_status fslbm_refill_scheme(fslbm_ctx *ctx, int32_t scheme);

/* Enable (1) or disable (0) replaying the step sequence as a captured HIP
 * graph (default: enabled).  The same kernels run either way; results are
 * bit-identical but where floating-point atomic sums (the bubble model's
 * per-bubble sums, the excess-mass reservoir) add in another order. */
fslbm_status fslbm_use_graphs(fslbm_ctx *ctx, int32_t enable);

/* Change the stream used by later calls (hipStream_t). */
fslbm_status fslbm_set_stream(fslbm_ctx *ctx, void *stream);

/*
 * Copy the canonical state into caller device buffers.  dst[k] is the
 * destination of field bit k (FSLBM_FIELD_*) and is only read when that bit is
 * set in field_mask; layouts as in the header comment.  Synchronises.
 * The reservoir scalar is returned by fslbm_diagnostics.
 */
fslbm_status fslbm_read_fields(fslbm_ctx *ctx, uint32_t field_mask, void *const *dst);

/* Per-domain diagnostics into the HOST array out[B].  Synchronises.  Returns
 * FSLBM_EUNSTABLE (without poisoning the context) if some domain holds
 * non-finite values or a speed above c_s = 1/sqrt(3) (the stability criterion
 * of Sec. 4). */
fslbm_status fslbm_diagnostics(fslbm_ctx *ctx, fslbm_diag *out);

/* Conversion activity of the most recent step, summed over all domains. */
typedef struct fslbm_step_stats {
    int64_t interface_cells;  /* interface cells after the step                  */
    int64_t new_from_gas;     /* gas cells that became interface (refilled)      */
    int64_t from_liquid;      /* liquid cells that became interface              */
    int64_t converted;        /* interface cells that became liquid or gas       */
} fslbm_step_stats;

/* Fill *out with the conversion activity of the last step (zeros before the
 * first step).  Synchronises. */
fslbm_status fslbm_last_step_stats(fslbm_ctx *ctx, fslbm_step_stats *out);

/*
 * Reverse mode: an interface-height loss over a window of T steps and its
 * gradient.  The paper does not differentiate the method; this is the adjoint
 * of the step (a), (b), (d) and (e) above, taken with the sequence of cell
 * types (and so every conversion decision) held fixed at what the forward run
 * produced.  Per domain b,
 *     L_b = (1/T) sum_{t=1..T} (h_b(t) - h*_b(t))^2,
 *     h_b(t) = sum of the fill level phi(t) over the cells with x = x_probe.
 * Differentiated quantities: omega_b, g_b, and the canonical state the window
 * starts from (f*, m, phi).  The reservoir of excess mass is part of the state
 * and is differentiated through.
 * Supported configuration: FSLBM_F64 storage, FSLBM_SRT, sigma = 0 and
 * FSLBM_REFILL_EQ (each call returns FSLBM_EINVAL otherwise); batch <= 65535.
 * Memory: sqrt(T)-style checkpointing.  The forward keeps K states; the
 * backward recomputes one segment of ceil(T/K) steps at a time from its
 * checkpoint and runs the reverse steps over it.
 */
typedef struct fslbm_adjoint_spec {
    int32_t nsteps;          /* T >= 1 steps in the window                          */
    int32_t n_checkpoints;   /* K in [1, T] stored states; 0 selects ceil(sqrt(T))  */
    int32_t x_probe;         /* probe plane, 0 <= x_probe < nx                      */
    int32_t pad;
    const double *target;    /* DEVICE [B][T]: h*_b(t) for t = 1..T; read by both   */
                             /* calls, so it must stay valid until the backward     */
} fslbm_adjoint_spec;

/* Bytes of the separate device workspace (256-byte aligned, owned by the
 * caller) that fslbm_adjoint_forward / _backward need for this spec. */
fslbm_status fslbm_adjoint_workspace_bytes(fslbm_ctx *ctx, const fslbm_adjoint_spec *spec,
                                           size_t *bytes);

/*
 * Run the T steps of the window from the context's current state, storing the
 * checkpoints in `workspace`.  loss: HOST [B] receives L_b.  height: HOST
 * [B][T+1] receives h_b(0..T), or NULL.  Synchronises.  Afterwards the context
 * holds the state at the end of the window.  Every checkpoint is written out
 * and read back, and the run continues from what was read, so the forward run
 * and the backward's recomputation produce bit-identical states.
 */
fslbm_status fslbm_adjoint_forward(fslbm_ctx *ctx, const fslbm_adjoint_spec *spec, void *workspace,
                                   size_t bytes, double *loss, double *height);

/*
 * Gradient of sum_b dloss[b] * L_b for the window of the last
 * fslbm_adjoint_forward on this context (same spec and workspace).
 *   dloss         HOST [B], or NULL for all ones.
 *   grad_omega    HOST [B]      dL/d omega_b.
 *   grad_gravity  HOST [B][3]   dL/d g_b.
 *   grad_pdf0     DEVICE [B][19][N] dL/d f*(x, start) (0 in gas), or NULL.
 *   grad_mass0    DEVICE [B][N]  dL/d m(x, start) (0 off the interface), or NULL.
 *   grad_phi0     DEVICE [B][N]  dL/d phi(x, start) (0 off the interface), or NULL.
 * May be called again with another dloss.  Synchronises.  Afterwards the
 * context holds the state at the end of the window again.
 */
fslbm_status fslbm_adjoint_backward(fslbm_ctx *ctx, const fslbm_adjoint_spec *spec, void *workspace,
                                    size_t bytes, const double *dloss, double *grad_omega,
                                    double *grad_gravity, double *grad_pdf0, double *grad_mass0,
                                    double *grad_phi0);

/* Text of the first error seen by this context (or by the last failed init
 * when ctx is NULL).  Never NULL. */
const char *fslbm_last_error(const fslbm_ctx *ctx);

/* Release the host-side context.  Does not touch the caller's workspace. */
void fslbm_destroy(fslbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FSLBM_H */
