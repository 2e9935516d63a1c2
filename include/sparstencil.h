/*
 * sparstencil -- stencil sweeps on gfx950 recast as 2:4-structured-sparse
 * matrix products (SparStencil, arXiv 2506.22969).
 *
 * C ABI of libsparstencil.so.  Every entry point takes plain host values and
 * host or device pointers, never throws, and reports failures through its
 * return code.  Device pointers are HIP device allocations on the current
 * device; `stream` arguments are hipStream_t values passed as void* (NULL =
 * the null stream).
 *
 * The operation: a fixed-coefficient stencil applied T times to a 1-, 2- or
 * 3-D grid (paper Section 2.2, with the commented Box-2D9P pseudo-code that
 * writes each sweep to a second mesh and swaps the meshes).  Sweep:
 *     out[p] = sum over the (2r+1)^d box offsets o of  w[o] * in~[p - r + o]
 * (correlation orientation), where in~ is `in` inside the grid and 0 outside
 * it (zero halo) or `in` at the index taken modulo the grid size (periodic).
 *
 * Grids are dense, row-major, slowest dimension first.  Split-state grids
 * hold their planes back to back: SS_SPLIT_BF16 [hi (N values) | lo (N)],
 * value = hi + lo; SS_SPLIT3_BF16 [hi | mid | lo], value = hi + mid + lo.
 */
#ifndef SPARSTENCIL_H
#define SPARSTENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SS_OK = 0,
    SS_PENDING = 1,          /* poll: job admitted or queued, not finished   */
    SS_E_INVALID = -1,       /* bad argument (null, size, shape, coeffs)     */
    SS_E_UNSUPPORTED = -2,   /* valid request no engine here implements      */
    SS_E_NOMEM = -3,         /* device or arena memory exhausted             */
    SS_E_DEVICE = -4,        /* a HIP call failed                            */
    SS_E_NOT_FOUND = -5,     /* unknown job id                               */
    SS_E_BUSY = -6           /* resource in use (e.g. job table full)        */
} ss_status;

/* Stencil shapes (paper Section 2.2: star and box patterns; the evaluation
 * of Section 4 spans kernels of other patterns too).  SS_SHAPE_CUSTOM: any
 * set of points in the (2r+1)^d box, given by the nonzero coefficients of
 * the box (sparstencil_plan) or as a list of offsets (sparstencil_plan_points). */
typedef enum { SS_SHAPE_BOX = 0, SS_SHAPE_STAR = 1, SS_SHAPE_CUSTOM = 2 } ss_shape;

/* State storage and arithmetic of a plan. */
typedef enum {
    SS_F64 = 0,            /* FP64 state, FP64 arithmetic                        */
    SS_F32 = 1,            /* FP32 state, FP32 arithmetic (direct engine)        */
    SS_F16 = 2,            /* binary16 state and coefficients, one binary16
                              product per K chunk accumulated in FP32, each
                              sweep's result rounded to binary16 (2-D matrix
                              engines; rows a multiple of 8 values)             */
    SS_F32_SPLIT_F16 = 3,  /* FP32 state; state and coefficients split into
                              binary16 hi + lo parts, products hi*hi + hi*lo +
                              lo*hi accumulated in FP32                         */
    SS_F32_SPLIT_BF16 = 4, /* as above with bfloat16 parts                       */
    SS_SPLIT_BF16 = 5,     /* state stored as bfloat16 hi and lo planes          */
    SS_SPLIT3_BF16 = 6     /* state stored as bfloat16 hi, mid and lo planes
                              (value = hi + mid + lo, 24 significant bits);
                              coefficients split into three bfloat16 parts;
                              products hi*hi, hi*mid, mid*hi, hi*lo, lo*hi and
                              mid*mid accumulated in FP32 (2-D matrix engines;
                              rows a multiple of 8 values)                     */
} ss_dtype;

typedef enum { SS_BC_ZERO = 0, SS_BC_PERIODIC = 1 } ss_boundary;

typedef enum {
    SS_ENGINE_AUTO = 0,    /* sparse MFMA where the plan supports it             */
    SS_ENGINE_SMFMAC = 1,  /* 2:4 sparse MFMA on the permuted staircase matrix   */
    SS_ENGINE_MFMA = 2,    /* dense MFMA on the unpermuted staircase matrix      */
    SS_ENGINE_DIRECT = 3   /* direct neighbour sum on the vector ALUs            */
} ss_engine;

typedef struct {
    uint32_t struct_size;  /* sizeof(ss_plan_opts)                               */
    int32_t boundary;      /* ss_boundary                                        */
    int32_t fuse_steps;    /* S >= 1 sweeps composed into one (at most 8):
                              periodic grids; with a zero halo, FP32-state
                              (split) grids only: 2-D with S = 2, or S = 3 at
                              radius 1; 3-D with S = 2 at radius 1; 1-D with
                              r*S <= 8.  The points within r(S-1) of an edge
                              are then recomputed exactly, in the sweep's
                              launch (a second launch on the 2-D direct
                              engine and for 2-D radii above 1)               */
    int32_t r1, r2;        /* tile width (x) and height (y); 0,0 = explore       */
    int32_t engine;        /* ss_engine                                          */
    uint32_t flags;        /* SS_FLAG_* bits, 0 by default                       */
} ss_plan_opts;

/* Build the host tables only: no device is touched, and run / sweep reject
 * the plan.  Lets tools and CPU tests read back plans without a GPU. */
#define SS_FLAG_HOST_ONLY 1u

typedef struct ss_plan_ *ss_plan_t;

/*
 * Build a plan (paper Sections 3.1-3.3: layout morphing, structured sparsity
 * conversion by Algorithm 1, layout exploration, metadata and lookup tables)
 * and upload its tables to the current device.
 *
 *   shape      SS_SHAPE_BOX, SS_SHAPE_STAR (coefficients 0 off the axes) or
 *              SS_SHAPE_CUSTOM (any pattern; planned as the box, the
 *              matrix-core K orders keeping only the columns it uses)
 *   radius     r >= 1
 *   coeffs     host, (2r+1)^ndim FP64 values, row-major, slowest dim first
 *   ndim       1, 2 or 3
 *   grid_dims  host, ndim sizes (slowest first), each >= 1
 *   dtype      ss_dtype
 *   opts       NULL for defaults (zero halo, S = 1, explore, auto engine)
 *
 * On success *out owns host and device tables until sparstencil_plan_destroy.
 * A plan is immutable and may be shared by threads.  Errors: SS_E_INVALID,
 * SS_E_UNSUPPORTED (e.g. no engine for the dtype/engine pair, a zero-halo
 * fusion outside the cases under fuse_steps, |coefficient| beyond the
 * binary16 range), SS_E_NOMEM, SS_E_DEVICE.  The matrix-core engines take
 * 2-D grids (FP32 split state, bfloat16 planes or plain binary16), 3-D grids (FP32 split
 * state) and 1-D grids (FP32 split state, tiles of 16 outputs, composed
 * radius up to 8); FP64 runs on MFMA for 2-D; the direct engine takes the
 * rest.
 */
ss_status sparstencil_plan(ss_plan_t *out, int32_t shape, int32_t radius, const double *coeffs,
                           int32_t ndim, const int64_t *grid_dims, int32_t dtype,
                           const ss_plan_opts *opts);

/*
 * Build a plan from a list of stencil points (SS_SHAPE_CUSTOM): point i has
 * offset offsets[i*ndim + d] along dimension d (slowest first) and
 * coefficient coeffs[i]; a sweep is out[p] = sum_i coeffs[i] * in~[p + o_i].
 * The plan is the one sparstencil_plan(SS_SHAPE_CUSTOM, r, W, ...) builds,
 * with r the largest |offset| component (1 for the centre alone) and W the
 * (2r+1)^ndim box holding coeffs[i] at offset o_i and 0 elsewhere.
 *   ndim       1, 2 or 3
 *   npoints    >= 1
 *   offsets    host, npoints * ndim int32 values; no offset twice, every
 *              component within [-16, 16]
 *   coeffs     host, npoints FP64 values
 * Other arguments, ownership and errors as for sparstencil_plan; a repeated
 * offset or one beyond radius 16 is SS_E_INVALID.
 */
ss_status sparstencil_plan_points(ss_plan_t *out, int32_t ndim, int32_t npoints, const int32_t *offsets,
                                  const double *coeffs, const int64_t *grid_dims, int32_t dtype,
                                  const ss_plan_opts *opts);

/* Plan read-back (for tests and tools).  Size protocol: with buf == NULL,
 * *nbytes receives the size; otherwise *nbytes must be >= the size and the
 * table is copied to host memory buf.  SS_E_INVALID for an unknown `what`. */
enum {
    SS_Q_INFO = 0,        /* ss_plan_info                                        */
    SS_Q_COEFFS = 1,      /* double[kf^ndim]: the (composed) coefficients used   */
    SS_Q_PERM = 2,        /* int32[K_pad]: A' column per K slot, -1 = zero col   */
    SS_Q_VALUES = 3,      /* double[m'][K_pad/2]: compressed A'' values          */
    SS_Q_META = 4,        /* uint8[m'][K_pad/4][2]: positions (i0 < i1)          */
    SS_Q_HI = 5,          /* uint16[m'][K_pad/2]: hi parts (bit patterns)        */
    SS_Q_LO = 6,          /* uint16[m'][K_pad/2]: lo parts, scaled by sigma      */
    SS_Q_MID = 11,        /* uint16[m'][K_pad/2]: mid parts (SS_SPLIT3_BF16;
                             empty otherwise)                                    */
    SS_Q_LUT = 7,         /* int32[K_pad][3]: (pz, pr, pc), -1s for zero cols    */
    SS_Q_MODEL = 8,       /* double[n][7]: r1, r2, T, T_compute, T_global,
                             T_shared, K_pad for every candidate layout          */
    SS_Q_KERNEL_LUT = 9,  /* int32[n]: LDS offsets the launched kernel gathers   */
    SS_Q_KERNEL_PERM = 10, /* int32[n]: A' column per K slot of the launched
                             matrix-core kernel, -1 = zero column: SS_Q_PERM's
                             groups with the columns the stencil never uses
                             dropped and re-paired (sparse), or the used column
                             pairs in natural order (dense); empty for the
                             direct engine                                        */
    SS_Q_KERNEL_FRAGS = 12 /* bytes: the launched matrix-core kernel's A
                             operand registers.  int32 {MB, KC, mode (0 sparse,
                             1 dense), parts (2, or 3 for SS_SPLIT3_BF16)},
                             then uint16 hi[MB][KC][64][8], lo[...] (and
                             mid[...] with 3 parts): lane l's eight 16-bit
                             values of M block MB, K chunk KC; sparse: then
                             uint32 idx[MB][KC][64], the 2-bit position of
                             value e within its 4-group at bits 2e+1:2e.
                             Sparse lane l holds row l % 16 and, for value e,
                             4-group 4*(2*((l/16)%2) + e/4) + 2*(l/32) +
                             (e/2)%2 of the chunk (K slots 4g .. 4g+3), two
                             values (e even, e odd) per group; dense lane l
                             holds row l % 16, K slots 8*(l/16) .. +7.  Empty
                             for the direct engine                           */
};

typedef struct {
    int32_t ndim, radius, k;          /* k = 2*radius_fused + 1               */
    int32_t fuse_steps;
    int32_t r1, r2, m_b, g, planes;
    int32_t m_prime, k_prime, k_pad, zeros;
    int32_t engine;                   /* engine actually used                 */
    int32_t dtype, boundary;
    int32_t passes;                   /* MMA passes per product (3 = split)   */
    int32_t launches_per_sweep;       /* kernel launches per (fused) sweep    */
    double sigma;                     /* lo-part scale (2^11 for binary16)    */
    double plan_seconds;              /* host time spent in sparstencil_plan  */
    int64_t dims[3];
} ss_plan_info;

ss_status sparstencil_plan_query(ss_plan_t plan, int32_t what, void *buf, size_t *nbytes);

/* Release a plan's host and device tables.  The caller must have finished
 * (synchronised) every run that uses it.  NULL is accepted. */
ss_status sparstencil_plan_destroy(ss_plan_t plan);

/*
 * Apply `steps` sweeps: the result is left in `out`.  Asynchronous on
 * `stream`; returns after enqueueing.
 *   in, out  device grids of the plan's dims and dtype (split: 2 planes);
 *            they must not overlap.  `in` serves as the second mesh of the
 *            ping-pong, so its contents are unspecified afterwards.
 *   steps    >= 0; 0 copies in to out.  With fuse_steps S > 1, floor(steps/S)
 *            fused launches run, then steps mod S unfused ones.  A 2-D
 *            FP64 grid of at most 2^20 points on the direct engine runs up
 *            to 16/r sweeps per launch (temporal blocking in LDS; each
 *            point's arithmetic as in single sweeps), so a run of at most
 *            16/r sweeps is one launch.
 * Errors: SS_E_INVALID (null, in == out, steps < 0), SS_E_DEVICE (launch).
 */
ss_status sparstencil_run(ss_plan_t plan, void *in, void *out, int64_t steps, void *stream);

/*
 * One (fused) sweep from `in` to `out` (no copy, no remainder handling): the
 * building block `run` repeats.  Same argument rules as sparstencil_run.
 */
ss_status sparstencil_sweep(ss_plan_t plan, const void *in, void *out, void *stream);

/*
 * One (fused) sweep of n grids of the plan's own dims and dtype in a single
 * launch (an ensemble of independent grids; each grid's result is
 * bit-identical to sparstencil_sweep of it alone).
 *   n        1..16
 *   in, out  host arrays of n device pointers; out[i] receives the sweep of
 *            in[i].  No output may overlap any input or another output.
 * Asynchronous on `stream`.  Errors: SS_E_INVALID (null, n out of range,
 * overlap, host-only plan), SS_E_DEVICE (launch).
 */
ss_status sparstencil_sweep_batch(ss_plan_t plan, int32_t n, const void *const *in, void *const *out,
                                  void *stream);

/* Number of kernels `run` launches for `steps` sweeps (0 for a copy); an
 * even count is preceded by one device-to-device copy of the grid. */
int64_t sparstencil_launch_count(ss_plan_t plan, int64_t steps);

/* Bytes of one grid buffer of the plan (all planes). */
size_t sparstencil_grid_bytes(ss_plan_t plan);

const char *sparstencil_status_string(int32_t status);

/*
 * Matrix-core throughput probe (measurement support, not part of the
 * method): launches `workgroups` workgroups of four waves, each wave running
 * `iters` rounds of 8 independent binary16 products on register operands
 * (SS_ENGINE_SMFMAC: v_smfmac_f32_16x16x64_f16; SS_ENGINE_MFMA:
 * v_mfma_f32_16x16x32_f16), then storing its accumulators to `out`.
 *   out    device buffer of workgroups * 256 * 4 floats (written)
 *   flops  host; receives the dense-equivalent flops the launch issues
 *          (2 * 16 * 16 * K per product, K = 64 sparse / 32 dense)
 * Asynchronous on `stream`: time it with events around the call.  Errors:
 * SS_E_INVALID (null, iters < 1, workgroups out of 1..2^20, other engine),
 * SS_E_DEVICE (launch).
 */
ss_status sparstencil_probe_mma_peak(int32_t engine, int64_t iters, int32_t workgroups, float *out,
                                     double *flops, void *stream);

/*
 * Serving loop (not part of the paper's method, which runs one grid at a
 * time: a batching layer around the sweep its Section 3.3 generates).  A server owns a
 * worker thread that admits submitted jobs first-come first-served while the
 * caller's device arena has room for a job's two buffers, then advances every
 * admitted job by one (fused) sweep per round.  Jobs whose plans have equal
 * device tables (same stencil, coefficients, dtype, boundary, fusion and
 * tile) are swept by one multi-grid launch per round, up to 16 grids; other
 * plan classes go to the server's other streams so their launches overlap.
 * A job's result is bit-identical to sparstencil_run of its plan.
 */
typedef struct ss_server_ *ss_server_t;

typedef struct {
    uint64_t id;
    int32_t state;         /* 0 queued, 1 running, 2 done, 3 failed             */
    int32_t status;        /* SS_OK, or the error that failed the job           */
    int64_t steps_total;   /* sweeps requested                                  */
    int64_t steps_done;    /* sweeps applied so far                             */
    double t_submit;       /* seconds on the server clock (sparstencil_server_clock) */
    double t_admit;        /* admitted into the arena (0 while queued)          */
    double t_done;         /* result copied to `out` (0 until then)             */
} ss_job_info;

/*
 * Create a server on the current device.
 *   arena        device memory the server sub-allocates job buffers from; the
 *                caller keeps ownership and frees it after destroy.
 *   arena_bytes  size of the arena.
 *   max_jobs     bound on queued + running jobs (submit returns SS_E_BUSY).
 *   num_streams  1..16 streams for concurrent plan classes.
 * Errors: SS_E_INVALID, SS_E_NOMEM, SS_E_DEVICE.
 */
ss_status sparstencil_server_create(ss_server_t *out, void *arena, size_t arena_bytes, int32_t max_jobs,
                                    int32_t num_streams);

/*
 * Queue `steps` (>= 1) sweeps of `plan` on the grid at `in`; the result is
 * written to `out` when the job finishes.  in and out may be host or device
 * memory and must stay valid, like the plan, until the job is done; `in` is
 * copied into the arena on admission and not modified.  *job_id receives the
 * job's id.  Errors: SS_E_INVALID (null, steps < 1, host-only plan, server
 * shutting down), SS_E_NOMEM (two grid buffers exceed the whole arena),
 * SS_E_BUSY (max_jobs reached).
 */
ss_status sparstencil_submit(ss_server_t server, ss_plan_t plan, const void *in, void *out, int64_t steps,
                             uint64_t *job_id);

/*
 * State of a job: SS_PENDING while queued or running, SS_OK when its result
 * is in `out`, the job's error if it failed, SS_E_NOT_FOUND for an unknown or
 * released id.  `info` (may be null) receives a snapshot.
 */
ss_status sparstencil_poll(ss_server_t server, uint64_t job_id, ss_job_info *info);

/* Forget a finished job's record (SS_E_BUSY while it is pending). */
ss_status sparstencil_job_release(ss_server_t server, uint64_t job_id);

/* Block until no job is queued or running. */
ss_status sparstencil_server_drain(ss_server_t server);

/* Seconds since the server was created (the clock of ss_job_info times). */
double sparstencil_server_clock(ss_server_t server);

/* Finish every queued and running job, then stop the worker and free the
 * server (not the arena).  A null server is a no-op. */
ss_status sparstencil_server_destroy(ss_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* SPARSTENCIL_H */
