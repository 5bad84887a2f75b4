/*
 * cglbm_serve.h -- continuous-batching solve server of the colour-gradient
 * LBM library (include/cglbm.h).
 *
 * Requests (independent lattices of any size and parameters) arrive through
 * lbm_enqueue_solve from any thread.  A server thread admits them in arrival
 * order as slots and device memory free up (HBM budget), keeps their
 * populations resident, and advances ALL active lattices with one kernel
 * launch per time step and group of lattices (the batched step of cglbm.h:
 * groups sized so that two fit the Infinity Cache together, two of them in
 * flight on two streams), in chunks of chunk_steps launches per group
 * replayed from captured HIP graphs.  A request that
 * needs fewer steps than a chunk stops at its own count (the kernel leaves
 * its lattice alone for the remaining launches).  Finished lattices are
 * retired at chunk boundaries (FP64 diagnostics, optional fields copied to
 * host memory, device memory released) and the freed capacity admits the
 * next arrivals.  Each lattice's arithmetic is exactly that of lbm_step:
 * a result is bit-identical whether the lattice ran alone or in a mix.
 *
 * Ownership: the server copies every input at enqueue; results stay in the
 * server until lbm_wait / lbm_poll return them (fields only if requested at
 * enqueue).  All functions are thread-safe.  Status codes as in cglbm.h.
 */
#ifndef CGLBM_SERVE_H
#define CGLBM_SERVE_H

#include "cglbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_server lbm_server;
typedef uint64_t lbm_req;

enum { LBM_INIT_FIELDS = 0, LBM_INIT_DISK = 1, LBM_INIT_BANDS = 2 };

/* Initial state of a request: the equilibrium (Sec. 2.1.1 eq. (equilibrium))
 * of sharp colour densities at rest, from host fields or a geometry. */
typedef struct {
    int32_t kind;                              /* LBM_INIT_*                                       */
    int32_t n_edges;                           /* BANDS: number of entries of edges                */
    const double *rho_r, *rho_b, *ux, *uy;     /* FIELDS: [ny][nx] (ux/uy may be NULL); copied     */
    double cx, cy, radius;                     /* DISK: node (x,y) is inside iff its cell centre   */
                                               /*   (x+1/2, y+1/2) lies strictly within radius     */
    double rho_r_in, rho_b_in;                 /* DISK: colour densities inside                    */
    double rho_r_out, rho_b_out;               /* DISK: colour densities outside                   */
    const int32_t *edges;                      /* BANDS: first columns of full-height bands,       */
                                               /*   edges[0] = 0, increasing; bands alternate       */
                                               /*   red (even) / blue (odd)                         */
    double rho_band_r, rho_band_b;             /* BANDS: density of a red band / of a blue band    */
    const int8_t *inlet_color;                 /* optional [ny] (+1 red, -1 blue); copied          */
} lbm_init_desc;

typedef struct {
    int32_t status;        /* LBM_OK, LBM_E_BUSY (not finished), LBM_E_UNSTABLE, LBM_E_NOMEM ... */
    int32_t slot;          /* slot index it ran in (-1 if never admitted)                       */
    int64_t steps_done;
    double t_arrive, t_admit, t_done;   /* seconds since the server was created                  */
    lbm_diag_t diag;       /* FP64 diagnostics of the final state; for a DISK request p_in and  */
                           /* p_out are the mean pressures at r < R - 4 and r > R + 4 around    */
                           /* (cx, cy), R = sqrt(area_r / pi) (Laplace sampling, Sec. 4)        */
    double *rho_r, *rho_b, *ux, *uy, *p; /* caller-owned [ny][nx] outputs, or NULL; filled when  */
                                         /* the request finished and was enqueued with fields   */
} lbm_result;

typedef struct {
    int64_t enqueued, admitted, completed, failed;
    int64_t chunks, launches;
    int64_t peak_active;
    uint64_t peak_bytes;        /* largest device memory held by active lattices             */
    double lattice_updates;     /* sum over finished work of nodes * steps                   */
    double busy_s;              /* time from chunk launch to chunk completion, summed         */
    double admit_s;             /* host time spent admitting (allocation, set-up, init)       */
    double retire_s;            /* host time spent retiring (diagnostics, fields, release)    */
} lbm_server_stats;

/* hbm_budget: device bytes the active lattices may hold in total (their
 * lbm_bytes_required); max_slots: lattices advanced together (<= 4096);
 * chunk_steps: launches per chunk (even, >= 2); storage: LBM_STORE_* used for
 * every request (a request's own storage field is ignored); tile_x: threads
 * per workgroup, 64, 128 or 256, or 0 for the launch planner's choice per
 * group of lattices; hip_stream: NULL for a server-owned stream. */
int lbm_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, int32_t storage,
                      int32_t tile_x, void *hip_stream, lbm_server **out);
/* The same scheduler with a host-only backend that performs no GPU work:
 * a chunk costs (lattice updates) / (mlups * 1e6) seconds of virtual time
 * and results carry only step counts.  For tests of the scheduling logic. */
int lbm_server_create_fake(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, double mlups,
                           lbm_server **out);
/* Non-blocking.  keep_fields: retain rho_r, rho_b, ux, uy, p of the final
 * state for lbm_wait / lbm_poll.  Invalid parameters are rejected here
 * (LBM_E_INVAL); a request larger than the whole budget finishes with
 * LBM_E_NOMEM. */
int lbm_enqueue_solve(lbm_server *s, const lbm_params *p, const lbm_init_desc *init, int64_t steps,
                      int32_t keep_fields, lbm_req *id);
/* LBM_E_BUSY while the request runs or waits; its final status when done;
 * LBM_E_NOTFOUND for an unknown id.  A finished request can be read again. */
int lbm_poll(lbm_server *s, lbm_req id, lbm_result *r);
int lbm_wait(lbm_server *s, lbm_req id, lbm_result *r);
/* Drop a finished request's stored result (fields included). */
int lbm_release(lbm_server *s, lbm_req id);
int lbm_server_stats_get(lbm_server *s, lbm_server_stats *st);
/* Test hook: the request fails (LBM_E_UNSTABLE) at its next chunk boundary. */
int lbm_server_inject_failure(lbm_server *s, lbm_req id);
/* Stops the server thread after the running chunk: queued requests are
 * dropped, running ones released, stored results freed.  No other call on
 * the server may be in progress or follow. */
int lbm_server_destroy(lbm_server *s);
const char *lbm_server_last_error(const lbm_server *s);

#ifdef __cplusplus
}
#endif
#endif
