/*
 * cglbm.h -- C ABI of the MI355X colour-gradient lattice Boltzmann library.
 *
 * Method: two-population colour-gradient LBM on D2Q9 (Douillet-Grellier,
 * Leclaire, Vidal, Bertrand, De Vuyst, arXiv:1903.01168, Sec. 2).  One time
 * step = pull streaming (Sec. 2 eq. (subop4)) with periodic wrap, halfway
 * bounce-back walls (Sec. 2.5 item 1) or two-phase Zou-He inlet/outlet
 * (Sec. 2.5 item 3), colour-blind BGK or MRT collision with omega interpolated
 * across the interface (Sec. 2.1.1-2.1.2), the surface-tension perturbation
 * (Sec. 2.2) and the recolouring (Sec. 2.3).  Everything runs in hand-written
 * HIP kernels for gfx950; host code only validates, plans and launches.
 *
 * General conventions
 *  - Every function returns an int status: LBM_OK (0) or a negative LBM_E_*
 *    code.  lbm_last_error(ctx) returns a message for the last failure on that
 *    context (ctx may be NULL for failures of the create functions; that
 *    message is per thread).  No C++ exception crosses this interface.
 *  - Host arrays are FP64, caller-owned, row-major [ny][nx] with x fastest and
 *    y pointing "north" (direction 2 of the lattice).
 *  - Velocity numbering: 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1);
 *    5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1) -- the order of the rows of the
 *    MRT matrix of Appendix B.
 *  - A context owns one lattice, is bound to one HIP stream and one device
 *    (the device current at creation), and is not thread-safe.  Calls on it
 *    are asynchronous on its stream unless stated otherwise.
 *  - The stored state is the population set after the recolouring of the last
 *    step, about to be streamed; the initial state is the equilibrium of the
 *    given fields.  "Fields at step n" are the moments of the streamed and
 *    boundary-completed populations, i.e. what step n+1 collides.
 */
#ifndef CGLBM_H
#define CGLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_E_INVAL (-1)    /* invalid argument or parameter combination        */
#define LBM_E_NOMEM (-2)    /* device or host allocation failed                  */
#define LBM_E_DEVICE (-3)   /* a HIP call failed (no device, launch failure ...) */
#define LBM_E_UNSTABLE (-4) /* non-finite values seen by the diagnostics         */
#define LBM_E_BUSY (-5)     /* request still running / capacity exhausted        */
#define LBM_E_NOTFOUND (-6) /* unknown request id                                */

/* Face boundary conditions.  x faces: both PERIODIC, or ZOUHE_VELOCITY on
 * x-low with ZOUHE_PRESSURE on x-high.  y faces: both PERIODIC, or walls
 * half-way outside the first/last row, each BOUNCEBACK (no slip: a population
 * that would come from beyond the wall is the node's own opposite one) or
 * FREESLIP (Sec. 2.5 item 1: diagonal populations are reflected forward along
 * the wall, i.e. a population that would come from beyond the wall is the
 * one with the opposite c_y that left the upstream node of the same row). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_BOUNCEBACK = 1, LBM_BC_ZOUHE_VELOCITY = 2, LBM_BC_ZOUHE_PRESSURE = 3,
       LBM_BC_FREESLIP = 4 };
enum { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };
/* Population storage.  Arithmetic is FP32 in every mode.  F32: 72 B per
 * node and buffer (9 red + 9 blue planes).  F16S / BF16S: for each moving
 * direction the colour-blind population N_i as a 16-bit (FP16 or BF16)
 * deviation (N_i - rho0_k phi^k_i) 2^12 / max(rho0_r, rho0_b) from the rest
 * state (the reference is the same for both fluids) and the red share
 * N^r_i / N_i as a 16-bit fixed-point fraction; the two rest populations in
 * FP32, each absorbing its node's exact colour-mass remainder; stochastic
 * rounding throughout.  40 B per node and buffer. */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16S = 1, LBM_STORE_BF16S = 2 };

typedef struct {
    int32_t nx, ny;                         /* lattice nodes, >= 1 (>= 2 along an open x) */
    int32_t bc_xlo, bc_xhi, bc_ylo, bc_yhi; /* LBM_BC_*                                   */
    int32_t collision;                      /* LBM_COLL_*                                 */
    int32_t storage;                        /* LBM_STORE_*                                */
    double rho0_r, rho0_b;   /* reference densities (> 0), Sec. 2.1.1                   */
    double alpha_light;      /* alpha of the lighter fluid, 0 < a < 1 (0.2 in the paper) */
    double tau_r, tau_b;     /* relaxation times (> 0.5); omega_k = 1/tau_k, Sec. 2.1.1  */
    double delta;            /* width of the omega interpolation (> 0; 0.1)              */
    double A;                /* perturbation amplitude, Sec. 2.2; or 0 with sigma > 0    */
    double sigma;            /* surface tension: A(x) = 9 sigma omega_eff(x) / 4 if > 0  */
    double beta;             /* recolouring parameter in [0, 1], Sec. 2.3                */
    double mrt_lambda;       /* s_0..s_6 = lambda omega_eff (0.8), Sec. 2.1.2            */
    double gx, gy;           /* body force per unit mass (Guo forcing)                   */
    double u_in_r, u_in_b;   /* inlet x-velocity of red / blue inlet nodes               */
    double p_out;            /* outlet pressure                                          */
    /* Static contact angle at y walls (Sec. 2.4): with wetting = 1, the colour
     * gradient of every node of the first and last row is turned, its length
     * kept, to the closer of the two directions that make the angle
     * 180 - contact_angle with the wall normal pointing into the fluid (the
     * gradient points into red, so contact_angle is the red fluid's angle,
     * measured through red; a tangential part of exactly 0 keeps the normal;
     * 0 and 180 turn every gradient onto the normal).  Needs y walls (either
     * kind).  wetting = 0 (zero-initialised struct): no adjustment, and
     * contact_angle is ignored. */
    int32_t wetting;         /* 0 or 1                                                   */
    int32_t reserved0;       /* must be 0                                                */
    double contact_angle;    /* degrees, 0 <= contact_angle <= 180                       */
    /* Navier-Stokes correction (Sec. 2.1.3; MRT only): ns_correction = 1 uses
     * the third-order Hermite equilibrium (its factor (3 c_i - 4) read as
     * (3 |c_i|^2 - 4)) in the collision, the initialisation and the Zou-He
     * completion (term H of Sec. 2.5 item 3), and adds the MRT source
     * M^-1 C with C_1 = 3 (1 - s_1/2)(dQx/dx + dQy/dy) and
     * C_7 = (1 - s_7/2)(dQx/dx - dQy/dy) (printed with a factor 3, omega_eff
     * and a plus sign; this form follows from row 7 of M, c_x^2 - c_y^2),
     * Q = sum_k (1.8 alpha_k - 0.8) rho_k u differentiated with the stencil
     * of eq. (colorGradient) (ghost values beyond walls and open faces as for
     * the colour field).  The kinematic viscosity of fluid k is then
     * c_s,k^2 (tau_k - 1/2) instead of (tau_k - 1/2) / 3. */
    int32_t ns_correction;   /* 0 or 1                                                   */
    int32_t reserved1;       /* must be 0                                                */
    /* Colour gradient: 0 = eq. (colorGradient), nearest neighbours; 1 = the
     * more isotropic operator the paper points to (Sec. 4): second
     * neighbours, 25 points, F = sum w(|c|^2) c psi(x + c) with w = 4/21,
     * 4/45, 1/60, 2/315, 1/5040 for |c|^2 = 1, 2, 4, 5, 8 (isotropic to 8th
     * order).  Beyond an open face the colour field takes the nearest column;
     * two rows beyond a wall it repeats the ghost row of Sec. 2.4; corner
     * cells beyond both repeat the inner ghost column.  Lower spurious
     * currents, more work per node. */
    int32_t gradient;        /* 0 or 1                                                   */
    int32_t reserved2;       /* must be 0                                                */
} lbm_params;

typedef struct {
    double mass_r, mass_b;   /* FP64 sums of rho_r and rho_b over the lattice            */
    double area_r;           /* sum of (1 + psi) / 2: volume of the red fluid            */
    double max_u;            /* max |u|                                                  */
    double p_in, p_out;      /* mean pressure for r < r_in and r > r_out (see lbm_diag)  */
    int64_t n_in, n_out;     /* node counts of those two regions                         */
    int64_t n_nonfinite;     /* nodes with a non-finite density or velocity              */
    int64_t step;            /* steps done                                               */
} lbm_diag_t;

typedef struct lbm_ctx lbm_ctx;

const char *lbm_version(void);
const char *lbm_last_error(const lbm_ctx *ctx);

/* Device bytes a context needs for these parameters: two population buffers
 * plus the field staging area.  Returns 0 for invalid parameters. */
size_t lbm_bytes_required(const lbm_params *p);
/* Bytes of one population buffer (both colours; row pitch padded to 64
 * nodes; 72 B per node in F32, 40 B with 16-bit storage). */
size_t lbm_buffer_bytes(const lbm_params *p);

/* Create a context on the current device.  hip_stream: a hipStream_t, or NULL
 * for a stream owned by the context.  Device memory is allocated here. */
int lbm_create(const lbm_params *p, void *hip_stream, lbm_ctx **out);
/* Same, with two caller-owned device buffers of lbm_buffer_bytes(p) bytes
 * each (256-byte aligned); they must outlive the context. */
int lbm_create_ext(const lbm_params *p, void *hip_stream, void *buf_a, void *buf_b,
                   size_t bytes_each, lbm_ctx **out);
int lbm_destroy(lbm_ctx *ctx);

/* Equilibrium initialisation (Sec. 2.1.1 eq. (equilibrium)) from host fields;
 * ux / uy may be NULL (zero).  Resets the step counter. */
int lbm_init_fields(lbm_ctx *ctx, const double *rho_r, const double *rho_b, const double *ux,
                    const double *uy);
/* Inlet colour per row (+1 red, -1 blue), for LBM_BC_ZOUHE_VELOCITY (Sec. 2.5
 * item 3).  Default: all red.  Takes effect for steps launched afterwards. */
int lbm_set_inlet_color(lbm_ctx *ctx, const int8_t *color_y);

/* Advance n >= 0 steps (asynchronous).  Long runs replay a captured HIP graph
 * of a fixed number of steps. */
int lbm_step(lbm_ctx *ctx, int64_t n);
int64_t lbm_steps_done(const lbm_ctx *ctx);
int lbm_sync(lbm_ctx *ctx);

/* Fields at the current step into caller-owned host arrays (any may be NULL):
 * the moments the next collision sees, i.e. of the populations each node
 * pulls from its neighbours after bounce-back and open-boundary completion
 * (Sec. 2 eq. (subop4), Sec. 2.5), with the half-force velocity shift;
 * p = sum_k rho_k c_s,k^2 (Sec. 2.1.1 eq. (pressureRelation)).  d (nullable)
 * receives the FP64 diagnostics without the pressure regions.  Synchronises;
 * returns LBM_E_UNSTABLE if a non-finite value was seen. */
int lbm_moments(lbm_ctx *ctx, double *rho_r, double *rho_b, double *ux, double *uy, double *p,
                lbm_diag_t *d);
/* FP64 diagnostics computed on the device (deterministic reduction order).
 * circle (nullable) = {cx, cy, r_in, r_out}: the mean pressure is taken over
 * nodes whose cell centre (x+1/2, y+1/2) lies at r < r_in and r > r_out. */
int lbm_diag(lbm_ctx *ctx, const double *circle, lbm_diag_t *d);
/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid it): lbm_diag with
 * its reduction scratch -- per-block FP64 partial sums and the final sums --
 * in a fixed per-device array of the library (147 528 bytes, 2048 blocks of
 * partials, held by each GPU the library runs on until the process ends)
 * instead of the context's work buffers.  Same kernels, same block count and
 * order, so the same bits as lbm_diag.  Allocates nothing; copies the nine
 * sums to the host and synchronises the context's stream.  All calls on one
 * GPU share that array: calls that overlap on one GPU (several threads or
 * streams) race.  Errors: as lbm_diag; LBM_E_INVAL if the lattice needs more
 * reduction blocks than the array holds (never, with the current block cap). */
int lbm_diag_noalloc(lbm_ctx *ctx, const double *circle, lbm_diag_t *d);

/* Populations of the stored state, decoded to FP64, layout [2][9][ny][nx]
 * (colour, direction, y, x); and the reverse (encoded to the storage type). */
int lbm_get_pops(lbm_ctx *ctx, double *host);
int lbm_set_pops(lbm_ctx *ctx, const double *host);

/* Raw checkpoint of the stored state (bit-exact resume): header + both colour
 * population planes in the storage format + the step counter.  *written
 * receives the size; with host == NULL only the size is returned. */
int lbm_save_state(lbm_ctx *ctx, void *host, size_t cap, size_t *written);
int lbm_load_state(lbm_ctx *ctx, const void *host, size_t n);

/* Launch-shape control (tuning): threads per workgroup (64, 128, 256, 512 or
 * 1024: one to sixteen wavefronts side by side; 0 = planned) and rows per
 * workgroup strip (0 = planned).  Results do not depend on either. */
int lbm_set_launch(lbm_ctx *ctx, int32_t tile_x, int32_t strip_rows);
/* Step-kernel flavour (tuning; nearest-neighbour gradient only -- the
 * second-neighbour gradient always uses halo lanes): 1 = block exchange (each
 * wavefront writes a whole 64-column block, edge columns exchanged through
 * LDS and the workgroup's outer halo nodes gathered beside each row: whole
 * cache lines written, for lattices beyond the last-level cache), 0 = halo
 * lanes (each wavefront writes 60 columns and its outer lanes hold the
 * neighbour columns), -1 = planned (block exchange for FP32 storage without
 * the Navier-Stokes correction when both population buffers exceed 256 MiB).
 * Results do not depend on it.
 * Errors: LBM_E_INVAL for another mode. */
int lbm_set_exchange(lbm_ctx *ctx, int32_t mode);
/* The HIP stream of the context (a hipStream_t). */
void *lbm_stream(const lbm_ctx *ctx);

/* ---- batched stepping -------------------------------------------------
 * A batch advances several contexts (same device, same storage type) with one
 * kernel launch per group of lattices and time step: every workgroup finds
 * its lattice in a device table of lattice descriptors.  A batch of two or more lattices is split
 * into groups (contiguous, balanced by bytes, at least two, never mixing
 * kernel variants) sized so that two groups fit MI355X's 256 MB Infinity
 * Cache together (240 MiB), and lbm_batch_step advances two groups at a time
 * on two streams of its own (rounds of 256 steps per group, the work of a
 * round halved between the streams; one group's launch then fills the chip
 * while the other's last wavefronts finish).  The streams start after the
 * work already queued on hip_stream and on the contexts' streams, and those
 * streams wait for them at the end of the call (no host synchronisation);
 * after the call every context has advanced n steps.  Each lattice's
 * arithmetic is exactly that of lbm_step, so results are bit-identical to
 * stepping the contexts one by one, in any grouping.  The contexts must not
 * be stepped outside the batch while it exists (LBM_E_INVAL otherwise);
 * lbm_moments / lbm_diag / checkpoints on them stay valid.  tile_x: threads
 * per workgroup, 0 (planned per group), 64, 128, 256, 512 or 1024.  Each
 * group's step flavour is planned (lbm_set_exchange: block exchange for FP32
 * groups without the Navier-Stokes correction whose two buffers exceed
 * 256 MiB). */
typedef struct lbm_batch lbm_batch;
int lbm_batch_create(lbm_ctx *const *ctxs, int32_t n, int32_t tile_x, void *hip_stream, lbm_batch **out);
int lbm_batch_step(lbm_batch *b, int64_t n);
int lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);
/* Number of cache-sized groups of the batch, i.e. kernel launches per step
 * (0 for a NULL batch). */
int lbm_batch_groups(const lbm_batch *b);
/* Launch shape of group g (0 <= g < lbm_batch_groups): threads per workgroup
 * and step flavour (1: block exchange, 0: halo lanes; see lbm_set_exchange).
 * Either pointer may be NULL.  Errors: LBM_E_INVAL for a NULL batch or a
 * group out of range. */
int lbm_batch_group_launch(const lbm_batch *b, int32_t g, int32_t *tile_x, int32_t *exchange);

/* Plain device-to-device copy of n bytes on the context stream (measures
 * achievable HBM bandwidth beside the step). */
int lbm_bw_copy(lbm_ctx *ctx, void *dst, const void *src, size_t n);

#ifdef __cplusplus
}
#endif
#endif
