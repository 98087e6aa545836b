/*
 * pct.h -- C ABI of the MI355X (gfx950) proton-CT reconstruction hot path.
 *
 * The problem (Karbasi et al., "A Highly Accelerated Parallel Multi-GPU based
 * Reconstruction Algorithm for Generating Accurate Relative Stopping Powers",
 * Section I): protons are tracked on entry to and exit from the object; each
 * proton's most likely path (MLP) through the voxel grid gives one sparse row
 * a_i of A (the chord length of the path in every voxel), b_i is its measured
 * water-equivalent path length (WEPL) and x the relative stopping power (RSP)
 * of every voxel.  A x = b is solved iteratively (Section III) with the
 * block-iterative DROP method, one block being the protons processed in
 * parallel (Section IV-B).
 *
 * The paper cites the MLP and DROP formulas without printing them.  This
 * library implements:
 *   MLP   -- the maximum-likelihood path of Schulte et al. (Med. Phys. 35,
 *            2008) between two fixed tracker planes u_in < u_out of the beam
 *            frame, sampled every `step` mm; the path is the polyline through
 *            those vertices;
 *   row   -- Siddon's ray/grid intersection on every polyline segment, voxel
 *            of a piece from its midpoint, half-open voxels; a_ij is the sum
 *            of the chords of the path inside voxel j;
 *   DROP  -- for every block t of B consecutive protons (input order),
 *            rho_i = lambda (b_i - a_i.x) / ||a_i||^2 and
 *            x_j += (sum_i rho_i a_ij) / s_j, s_j = number of block rows that
 *            touch voxel j; rows with ||a_i|| = 0 are skipped.
 *
 * Frames and units.  Lab frame (x, y, z) in mm.  Voxel (ix, iy, iz) covers
 * [origin + i*pitch, origin + (i+1)*pitch) on each axis and has flat index
 * j = ix + nx*(iy + ny*iz).  At gantry angle phi the beam frame is
 * e_u = (cos phi, sin phi, 0), e_t = (-sin phi, cos phi, 0), e_v = (0, 0, 1);
 * a tracker measurement (t, v, th, ph) is a lateral position (mm) and the
 * slopes dt/du, dv/du.
 *
 * Memory.  Every data pointer passed to a compute call (proton arrays, b, x,
 * y, r, g, trace outputs, the workspace) is DEVICE memory owned by the
 * caller.  The library allocates no device memory: all scratch lives in a
 * caller-provided workspace of pct_workspace_size() bytes, which must first
 * be initialised by pct_plan_upload().  Calls are asynchronous on `stream`
 * (a hipStream_t; NULL is the null stream); results are valid once the caller
 * synchronises that stream.
 *
 * Errors.  Every call returns PCT_OK (0) or a negative status.  All argument
 * checks run on the host before anything is enqueued, so a call that returns
 * an argument error has launched nothing.  Conditions only the device can see
 * (a row longer than the caller's trace buffer, a re-entry pattern outside the
 * kernel's window, non-finite inputs) are recorded in a status word inside
 * the workspace and read back with pct_device_status().
 */
#ifndef PCT_H
#define PCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PCT_OK 0
#define PCT_ERR_INVALID_ARG (-1)   /* a pointer, size, geometry or option is invalid     */
#define PCT_ERR_WORKSPACE (-2)     /* workspace missing, too small or not uploaded        */
#define PCT_ERR_ROW_OVERFLOW (-3)  /* (device) a traced row exceeded max_nnz              */
#define PCT_ERR_NONFINITE (-4)     /* (device) a proton record or b_i was NaN/Inf        */
#define PCT_ERR_REENTRY (-5)       /* (device) a voxel re-entry outside the kernel window */
#define PCT_ERR_HIP (-6)           /* a HIP runtime call failed (see pct_last_hip_error)  */
#define PCT_ERR_UNSUPPORTED (-7)   /* valid request this build does not implement         */
#define PCT_ERR_CANCELLED (-8)     /* (device) a cancellable DROP call stopped on request */

/* device status bits returned by pct_device_status() */
#define PCT_DEV_ROW_OVERFLOW 0x1u
#define PCT_DEV_NONFINITE 0x2u
#define PCT_DEV_REENTRY 0x4u
/* FP32 DROP: a contribution |rho_i a_ij| reached 2^12 (it is clamped to
 * +-2^12; a NaN one counts as 0), or, on the binned schedule, the sum over a
 * block's rows of their largest contribution reached 2^15, the bound past
 * which a voxel's block sum may leave the +-2^15 range of the packed
 * fixed-point word (sums are not checked one by one: x is exact only if none
 * actually left it; the atomic schedules do not form this bound).  Use the
 * FP64 value type, a smaller B or a smaller lambda for such data. */
#define PCT_DEV_ACC_RANGE 0x8u
#define PCT_DEV_BAD_ROW 0x10u  /* a stored row names a voxel outside the plan's grid (piece skipped) */
#define PCT_DEV_CANCELLED 0x20u /* a cancellable DROP call stopped at a block boundary on request */

/* ---- value and chord types --------------------------------------------- */
typedef enum {
    PCT_F32 = 0, /* float  */
    PCT_F64 = 1  /* double */
} pct_dtype;

/* Precision of the chord lengths a_ij used by the solver.  Chords are always
 * computed in FP64; F32/F16/BF16 round each merged chord to FP32 and then to
 * the narrower format (round to nearest, ties to even) before any use. */
typedef enum {
    PCT_CHORD_F64 = 0,
    PCT_CHORD_F32 = 1,
    PCT_CHORD_F16 = 2,
    PCT_CHORD_BF16 = 3
} pct_chord;

/* ---- geometry and model ------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nz; /* voxels per axis, each > 0, nx*ny*nz < 2^31              */
    double pitch[3];    /* voxel size per axis (mm), > 0                           */
    double origin[3];   /* lab coordinates of the grid's minimum corner (mm)       */
} pct_grid;

typedef struct {
    double u_in, u_out; /* tracker planes along the beam axis (mm), u_in < u_out   */
    double step;        /* MLP vertex spacing in depth (mm), > 0                   */
    double poly[6];     /* 1/(beta^2 p^2) = sum_k poly[k] s^k [MeV^-2], s = depth
                           from u_in in cm                                          */
    double E0;          /* Highland constant (MeV), > 0                            */
    double X0;          /* radiation length (cm), > 0                              */
    int32_t log_term;   /* 1: scattering matrices carry (1 + 0.038 ln(L/X0))^2     */
} pct_mlp;

/* Structure-of-arrays proton records, n entries each, float32 device arrays. */
typedef struct {
    const float *t_in, *v_in;   /* entry lateral positions (mm) at u_in          */
    const float *th_in, *ph_in; /* entry slopes dt/du, dv/du                      */
    const float *t_out, *v_out; /* exit lateral positions (mm) at u_out          */
    const float *th_out, *ph_out;
    const float *gantry;        /* gantry angle phi (rad)                         */
    int64_t n;                  /* number of protons, >= 0                        */
} pct_protons;

/* Writable SoA proton arrays of `capacity` records (device memory). */
typedef struct {
    float *t_in, *v_in, *th_in, *ph_in, *t_out, *v_out, *th_out, *ph_out, *gantry;
    int64_t capacity;
} pct_protons_buf;


/* ---- plan --------------------------------------------------------------- */
/* Host object holding the grid, the MLP model and its FP64 coefficient table
 * (one row per vertex: t_k = c0t t_in + c0th th_in + c2t t_out + c2th th_out).
 * Its geometry is fixed after pct_plan_create (pct_plan_set_hull aside, which
 * needs no work in flight).  Calls on different threads and streams may share
 * a plan as long as each uses its own workspace: pct_drop_iterate and
 * pct_drop_iterate_rows keep a per-plan cache (the HIP graph of the last
 * sweep, re-recorded when the call's buffers or options change, and the
 * profiling events), and the plan's lock serialises their host-side enqueue;
 * their device work on different streams may overlap.  pct_profile_read
 * reports the last profiled call of any thread. */
typedef struct pct_plan pct_plan;

int pct_plan_create(const pct_grid *grid, const pct_mlp *mlp, pct_plan **out);
void pct_plan_destroy(pct_plan *plan);

/* Object hull: the z-cylinder (x - cx)^2 + (y - cy)^2 < radius^2, lab mm. */
typedef struct {
    double cx, cy, radius;
} pct_hull;

/* Per-proton paths through a hull (Section I: the MLP is evaluated from where
 * the proton enters the object to where it leaves it).  With hull != NULL
 * every row is the straight entry track from the entry tracker plane to the
 * hull, the most likely path between the points where the entry and exit
 * tracks meet the hull (its own depth D, polynomial depth measured from the
 * hull entry, vertices every `step` mm), and the straight exit track to the
 * exit tracker plane; a track pair that does not cross the hull gives one
 * straight segment between the tracker points.  Hull crossings outside the
 * tracker planes are clamped to them.  NULL restores the tracker-to-tracker
 * MLP of the shared table.  Host only; no work using the plan may be in
 * flight.  radius must be finite and > 0, the centre finite. */
int pct_plan_set_hull(pct_plan *plan, const pct_hull *hull);

/* Number of polyline segments K (vertices 0..K). */
int pct_plan_segments(const pct_plan *plan, int32_t *K);

/* Copies the host coefficient table, (K+1) rows of (c0t, c0th, c2t, c2th), into
 * host memory `tab` of (K+1)*4 doubles. */
int pct_plan_table(const pct_plan *plan, double *tab, int64_t tab_len);

/* DROP options. */
typedef struct {
    int64_t block;       /* protons per block B, > 0                                */
    double lambda;       /* relaxation, finite, > 0                                 */
    int32_t n_iter;      /* sweeps over all blocks, >= 0                            */
    int32_t dtype;       /* pct_dtype of x.  FP64: FP64 block accumulator and count;
                            FP32: one 64-bit word per voxel with the row count and
                            the block sum in 2^-28 fixed point (order-independent,
                            so results are bitwise reproducible); the block sum of
                            a voxel must stay below 2^15 in magnitude: see
                            PCT_DEV_ACC_RANGE                                      */
    int32_t chord;       /* pct_chord                                               */
    uint32_t flags;      /* PCT_DROP_* bits                                         */
    int64_t block_begin; /* first block of every sweep (>= 0)                       */
    int64_t block_end;   /* one past the last block; < 0 means ceil(n/B)            */
    int32_t lanes;       /* lanes per proton in the block kernel: 0 automatic, or
                            1, 8, 16, 32, 64                                         */
    int32_t reserved;    /* must be 0                                              */
} pct_drop_opts;

#define PCT_DROP_CHECK_FINITE 0x1u /* reserved: records and b are always checked      */
/* B must be below 2^19 (the packed count field) for the FP32 value type. */
#define PCT_DROP_NO_GRAPH 0x2u     /* launch per block on the stream, no HIP graph   */
#define PCT_DROP_PROFILE 0x4u      /* bracket a sample of the per-block kernels with
                                      HIP events on `stream` (see pct_profile_read) */
/* Block schedules of the FP32 value type with lanes > 1 (DROP's block step,
 * Section IV-B: all rows of block t against the same iterate, then the
 * D-weighted back-projection committed before block t+1).
 *
 * Default, when the workspace holds the slab bins of B rows (pct_workspace_size
 * with n >= B) and max(nx, ny) <= 8192: the binned schedule.  Per block, one
 * launch walks the rows and stores each lane's packed contributions (row count
 * bit + fixed-point rho_i a_ij) into per-(slab, row) bins of the block's
 * dominant in-plane axis; a second launch sums each slab's bins in LDS, one
 * workgroup per slab, and commits x_j += acc_j / s_j over exactly the touched
 * voxels.  The per-voxel integer sums equal those of the atomic schedules.
 * By default the commit carries the FP32 iterate's rounding error in a second
 * FP32 word per voxel (workspace, zeroed at the start of each call), so x is
 * rounded once per call rather than once per commit; the gathers read the
 * FP32 x.  Without a workspace large enough, the fused schedules below run. */
#define PCT_DROP_NO_COMPENSATION 0x40u /* binned schedule: round x at every commit
                                          (bitwise the atomic schedules' result) */
/* The atomic schedules: every piece is one 64-bit atomic into a packed
 * block accumulator.  Fused: the commit of block t-1 runs inside the launch
 * of block t (block t reads x + D * block sum of t-1, the value the commit
 * writes, so the result is bitwise that of the separate schedule). */
#define PCT_DROP_FUSED_COMMIT 0x20u
/* The separate schedule: one block kernel and one commit kernel per block
 * (also the FP64 value type's schedule). */
#define PCT_DROP_SEPARATE_COMMIT 0x8u
/* Fused schedule, 64 lanes per proton, blocks of at most 4096 protons,
 * workspace sized for the block: by default the rows of block t+1 are traced
 * in the launch that runs the DROP step of block t (the rows do not depend on
 * x), so each block step no longer waits for its own walk; results are
 * bitwise those of the other atomic schedules.  This flag asks for the plain
 * fused schedule. */
#define PCT_DROP_NO_TRACE_AHEAD 0x10u
/* Cancellable call: the block steps stop at the first block boundary after a
 * pct_drop_cancel request on this workspace (see there).  The call runs the
 * binned schedule when it would otherwise (FP32), else the separate schedule
 * (FP64, or FP32 without the bins' workspace); the fused and traced-ahead
 * atomic schedules, whose launches commit the previous block, are not used. */
#define PCT_DROP_CANCELLABLE 0x80u
/* Deterministic FP64 block sums: each contribution rho_i a_ij is split into
 * its bits above 2^-28 and the rest rounded at 2^-72, and both parts are
 * summed in 64-bit integers (two accumulator words per voxel), so FP64 runs
 * are bitwise reproducible whatever the order of the adds (the default FP64
 * schedule adds doubles with atomics, whose order varies).  A contribution of
 * 2^16 or more is clamped and raises PCT_DEV_ACC_RANGE; B must be below 2^19.
 * FP32 block sums are integers already: the flag changes nothing there. */
#define PCT_DROP_DETERMINISTIC 0x100u

/* Workspace bytes for this plan and x of type dtype.  n > 0 adds, for DROP
 * blocks of up to n protons, two row slots (the traced-ahead schedule,
 * 2 * n * 6.4 KB) and the slab bins of the binned schedule
 * (max(nx, ny) * n * 64 B + 2 * max(nx, ny) * n B); with n = 0 pct_drop_iterate
 * uses the atomic schedules. */
int pct_workspace_size(const pct_plan *plan, int64_t n, int32_t dtype, size_t *bytes);

/* Writes the coefficient table into the workspace and clears its counters and
 * status word.  Must precede every compute call that uses this workspace. */
int pct_plan_upload(pct_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Reads (and with reset != 0 clears) the device status word of the workspace;
 * synchronises `stream`.  *bits receives PCT_DEV_* flags. */
int pct_device_status(const pct_plan *plan, void *ws, size_t ws_bytes, int reset, uint32_t *bits, void *stream);

/* ---- entry points of the hot path -------------------------------------- */

/* Row tracing (MLP + voxel walk).  For protons first..first+count-1, writes the
 * ordered emission list of each path -- (voxel, chord) pieces in path order,
 * consecutive pieces in the same voxel merged -- to vox/chord rows of stride
 * max_nnz, and its full length to nnz.  Pieces beyond max_nnz are dropped and
 * PCT_DEV_ROW_OVERFLOW is raised.  vox: int32[count*max_nnz], chord:
 * double[count*max_nnz], nnz: int32[count]. */
int pct_mlp_trace(const pct_plan *plan, const pct_protons *p, int64_t first, int64_t count, int32_t max_nnz,
                  int32_t *vox, double *chord, int32_t *nnz, void *ws, size_t ws_bytes, void *stream);

/* Forward projection y = A x (and ||a_i||^2 if nrm2 != NULL).  x: dtype[nvox];
 * y, nrm2: dtype[n]. */
int pct_forward(const pct_plan *plan, const pct_protons *p, const void *x, int32_t dtype, void *y, void *nrm2,
                void *ws, size_t ws_bytes, void *stream);

/* Back projection g += A^T r.  r: dtype[n]; g: dtype[nvox], accumulated. */
int pct_backproject(const pct_plan *plan, const pct_protons *p, const void *r, int32_t dtype, void *g, void *ws,
                    size_t ws_bytes, void *stream);

/* Block-iterative DROP: opts->n_iter sweeps over blocks [block_begin,
 * block_end) updating x in place.  b: float[n]; x: dtype[nvox]. */
int pct_drop_iterate(const pct_plan *plan, const pct_protons *p, const float *b, void *x,
                     const pct_drop_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* Cancellation of DROP calls made with PCT_DROP_CANCELLABLE (a host-settable
 * request checked between block steps).  request != 0 asks the calls running
 * or queued on this workspace to stop: the block step whose commit sees the
 * request is the last one applied (x holds every block step before it, each
 * whole, and nothing after it; later sweeps of the call do nothing).  The
 * request stays until pct_drop_cancel(..., 0) clears it, so a cancellable
 * call started while it is set applies one block step.  The word is written
 * on a private stream of the plan and the call returns once it is written;
 * it does not wait for the DROP.  Calls without the flag ignore the request.
 * PCT_ERR_INVALID_ARG for a missing plan or workspace, PCT_ERR_WORKSPACE for
 * one that is too small, PCT_ERR_HIP if the write fails. */
int pct_drop_cancel(pct_plan *plan, void *ws, size_t ws_bytes, int32_t request);

/* Progress of the last cancellable DROP call on this workspace; synchronises
 * `stream` first.  *blocks_done receives the block steps it applied, counted
 * over all its sweeps (sweep s, block t of [block_begin, block_end) is step
 * s * (block_end - block_begin) + (t - block_begin) + 1).  Returns PCT_OK when
 * the call ran to its end, PCT_ERR_CANCELLED when it stopped on request; to
 * resume, run the rest of the interrupted sweep (block_begin moved past the
 * applied steps) and then the remaining sweeps. */
int pct_drop_progress(const pct_plan *plan, void *ws, size_t ws_bytes, int64_t *blocks_done, void *stream);

/* Smoothed total variation (differentiation form): TV(x) = sum_v sqrt(dx^2 +
 * dy^2 + dz^2 + eps^2) with forward differences, zero at the last index of
 * every axis.  Writes the value to value_dev (device double[1], summed in
 * FP64) and, if grad != NULL, its gradient.  x, grad: dtype[nvox]. */
int pct_tv(const pct_plan *plan, const void *x, int32_t dtype, double eps, double *value_dev, void *grad,
           void *ws, size_t ws_bytes, void *stream);

/* pct_tv for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * value and gradient, bitwise, with no workspace.  Its only scratch, the
 * per-workgroup partial sums (at most 4096 doubles, 32 KB, whatever the
 * grid), is a device array inside the library, one per GPU, held until the
 * process ends; it allocates nothing.  Calls that overlap on one GPU share
 * that array and race: serialise them (one stream per GPU, or events).  x,
 * value_dev and grad as for pct_tv; plan need not be uploaded.  Errors:
 * PCT_ERR_INVALID_ARG as pct_tv, PCT_ERR_HIP if the array's device address
 * cannot be found on the current device (at most 64 devices). */
int pct_tv_static(const pct_plan *plan, const void *x, int32_t dtype, double eps, double *value_dev, void *grad,
                  void *stream);

/* Within-block ordering.  Writes the records (and b, if not NULL) to out with
 * every block of `block` consecutive records sorted by (entry slice of v_in,
 * t_in, input position).  The DROP block update is a sum over the rows of the
 * block, so the order inside a block does not change it (with the FP32 value
 * type the block accumulator is order-independent and results are bitwise
 * equal); ordered blocks let the fused block kernel give each XCD a band of
 * neighbouring paths whose voxels stay in that XCD's L2.  Needs 1 <= block <=
 * 8192 and out->capacity >= p->n; out must not alias p.  Host-synchronous
 * validation, asynchronous on `stream`. */
int pct_order_blocks(const pct_plan *plan, const pct_protons *p, const float *b, int64_t block,
                     const pct_protons_buf *out, float *b_out, void *stream);

/* ---- angle-bin sort of acquisition-order scans (Section IV-A) -------------
 * The paper reconstructs a scan taken with continuous gantry rotation; its
 * records arrive in acquisition order.  pct_sort_scan groups them for the
 * block-iterative solve: a stable sort by the key (a, s, t_in) with
 *   a = floor(phi / dphi + 1/2) mod n_angles, dphi = 2 pi / n_angles, in FP64
 *       from the FP32 gantry angle (the angle bin of the FBP entry points);
 *   s = floor((v_in - z0) / slab_mm) in FP64, clamped to [0, n_slabs - 1],
 *       z0 the grid's lower z edge, n_slabs = ceil(nz pz / slab_mm);
 *   t_in compared as a number (-0 equals +0);
 * records with equal keys keep their input order, and a record whose gantry
 * angle, v_in or t_in is not finite goes after all others, in input order.
 * The result is unique (bit-exact whatever the launch shape).  Needs
 * 1 <= n_angles <= 4096, slab_mm > 0 and finite with n_slabs <= 4096,
 * reserved = 0. */
typedef struct {
    int32_t n_angles;
    int32_t reserved;   /* must be 0 */
    double slab_mm;
} pct_sort_opts;

/* Device workspace for pct_sort_scan on n records: 64 n bytes (keys,
 * positions and a packed copy of the records) plus about n / 2 bytes of
 * digit counts (256 per tile of 2048 records).  PCT_ERR_INVALID_ARG for
 * n < 0, n >= 2^31 or bytes == NULL. */
int pct_sort_scan_workspace_size(int64_t n, size_t *bytes);

/* Writes the records (and b, if not NULL) to out in the order above, and, if
 * perm is not NULL, perm[j] = input position of output record j (device
 * int64[n]).  Needs p->n < 2^31, out->capacity >= p->n, b_out when b is given;
 * out, b_out and perm must not alias the input or each other.  ws: device,
 * 256-byte aligned, at least pct_sort_scan_workspace_size(p->n) bytes, used
 * as scratch.  Host-synchronous validation (PCT_ERR_INVALID_ARG for bad
 * options or buffers, PCT_ERR_WORKSPACE for a missing, small or misaligned
 * workspace; nothing is launched then), asynchronous on `stream`. */
int pct_sort_scan(const pct_plan *plan, const pct_protons *p, const float *b, const pct_sort_opts *opts,
                  const pct_protons_buf *out, float *b_out, int64_t *perm, void *ws, size_t ws_bytes,
                  void *stream);

/* ---- stored rows (precision form) ----------------------------------------
 * The precision form lets the chord lengths be stored rather than recomputed.
 * With 288 GB of HBM the rows of the scans here fit (10^7 protons x ~257
 * pieces x 6 B = 15 GB with FP16 chords), so each row is traced once and the
 * DROP sweeps read it back.  Rows are CSR in device memory owned by the
 * caller: piece k of row i is at offsets[i] + k, in path order (the emission
 * list after consecutive merge); vox holds the voxel index, with bit 31 set
 * on the first piece of each distinct voxel of the row (so the row counts
 * once in s_j); chord holds the merged chord rounded to chord_type; n2 holds
 * ||a_i||^2 of the rounded row (re-entries summed per voxel first) in FP64. */
typedef struct {
    const int64_t *offsets; /* n + 1 */
    const int32_t *vox;     /* offsets[n] */
    const void *chord;      /* offsets[n] values: float (PCT_CHORD_F32) or FP16 / BF16 bit patterns (uint16) */
    const double *n2;       /* n */
    int64_t n;
    int32_t chord_type;     /* PCT_CHORD_F32, PCT_CHORD_F16 or PCT_CHORD_BF16 */
    int32_t reserved;       /* must be 0 */
} pct_rows;

/* Row lengths and their prefix sums: offsets[0] = 0, offsets[i+1] =
 * offsets[i] + (pieces of row i).  offsets: device int64[n+1]. */
int pct_rows_count(const pct_plan *plan, const pct_protons *p, int64_t *offsets, void *ws, size_t ws_bytes,
                   void *stream);

/* Traces every row into the CSR arrays laid out by pct_rows_count (vox:
 * int32[offsets[n]], chord: offsets[n] values of chord_type, n2: double[n]).
 * A row whose length differs from its offsets raises PCT_DEV_ROW_OVERFLOW
 * (pieces past its end are not written). */
int pct_rows_build(const pct_plan *plan, const pct_protons *p, int32_t chord_type, const int64_t *offsets,
                   int32_t *vox, void *chord, double *n2, void *ws, size_t ws_bytes, void *stream);

/* Block-iterative DROP over stored rows: as pct_drop_iterate, with the rows
 * read instead of traced.  FP32 x only (PCT_ERR_UNSUPPORTED otherwise);
 * opts->chord must equal rows->chord_type; opts->lanes: 0 (64), 16, 32 or 64
 * lanes per row; PCT_DROP_SEPARATE_COMMIT and PCT_DROP_CANCELLABLE are not
 * supported (PCT_ERR_UNSUPPORTED). */
int pct_drop_iterate_rows(const pct_plan *plan, const pct_rows *rows, const float *b, void *x,
                          const pct_drop_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* ---- multi-region reconstruction (Algorithm 1, Section III) --------------
 * The volume is cut along z into overlapping slab regions; each proton goes to
 * every region holding both its entry slice (of v_in) and its exit slice (of
 * v_out); every region is solved on its own (any entry point above, on a
 * region plan); each slice of the final image is taken from the region whose
 * core (non-overlapped part) holds it (selectSlice). */

/* Host only.  Region r of n_regions: core slices [core_lo[r], core_hi[r]] =
 * [floor(r nz / R), floor((r+1) nz / R) - 1]; region slices [z_lo[r],
 * z_hi[r]] = the core extended by `halo` slices past every interior core
 * boundary (the overlap of two neighbours is 2*halo slices).  Arrays of
 * n_regions int32 (host memory).  Needs 1 <= n_regions <= nz, halo >= 0. */
int pct_region_layout(int32_t nz, int32_t n_regions, int32_t halo, int32_t *z_lo, int32_t *z_hi, int32_t *core_lo,
                      int32_t *core_hi);

/* Host only.  A plan for slices z_lo..z_hi of the parent's grid (same x-y
 * extent, MLP model and hull setting, z origin moved up by z_lo slices). */
int pct_plan_region(const pct_plan *parent, int32_t z_lo, int32_t z_hi, pct_plan **out);

/* Step 2 of Algorithm 1 for one region: the records (and b) of the protons
 * whose entry and exit slices both lie in [z_lo, z_hi] of the plan's grid are
 * copied, in input order, to out (and b_out if b != NULL).  A slice is
 * floor((v - origin_z) / pitch_z) in FP64, clamped to [0, nz-1]; a record
 * with non-finite v_in or v_out belongs to no region.  *count (device
 * int64[1]) receives the number of members; records past out->capacity are
 * not written (compare *count with the capacity after synchronising). */
int pct_region_select(const pct_plan *plan, const pct_protons *p, const float *b, int32_t z_lo, int32_t z_hi,
                      const pct_protons_buf *out, float *b_out, int64_t *count, void *ws, size_t ws_bytes,
                      void *stream);

/* Coverage statistics of the proton tracks (the quantity of Table I, which
 * sets the overlap): hist[k] += number of protons whose entry and exit slices
 * (as in pct_region_select) differ by k, k = 0..nz-1; records with non-finite
 * v_in or v_out are not counted.  hist: device int64[nz], accumulated.
 * PCT_ERR_UNSUPPORTED for nz > 16384. */
int pct_slice_span_histogram(const pct_plan *plan, const pct_protons *p, int64_t *hist, void *ws, size_t ws_bytes,
                             void *stream);

/* selectSlice / region extraction: copies slices [z_first, z_first + z_count)
 * of the plan's grid from volume src, whose first slice is src_z0, to volume
 * dst, whose first slice is dst_z0 (x-y planes of nx*ny values of dtype).
 * Needs src_z0 <= z_first, dst_z0 <= z_first, z_first + z_count <= nz. */
int pct_select_slices(const pct_plan *plan, const void *src, int32_t src_z0, void *dst, int32_t dst_z0,
                      int32_t z_first, int32_t z_count, int32_t dtype, void *stream);

/* ---- FBP initial iterate (Section I) --------------------------------------
 * The iterative solve starts from a filtered back-projection (FBP) image.  The
 * paper does not print its FBP; this library implements parallel-beam FBP
 * slice by slice along each proton's straight entry-to-exit chord (Kak &
 * Slaney, Principles of Computerized Tomographic Imaging, ch. 3):
 *   binning  -- proton i goes to angle bin a = floor(phi / dphi + 1/2) mod
 *               n_angles (dphi = 2 pi / n_angles), lateral bin
 *               k = floor((t_c - t0) / dt) and the slice iz of the plan's grid
 *               holding v_c, (t_c, v_c) being the chord at depth u = 0:
 *               t_c = t_in + w (t_out - t_in), w = -u_in / (u_out - u_in), same
 *               for v.  Protons outside the bins, with a non-finite field or b,
 *               or with |b| >= 2^20 mm are dropped.  The projection of a bin
 *               is the mean b of its protons, 0 for an empty bin.  Sums are
 *               accumulated in 2^-24 mm fixed point (order-independent);
 *               a bin's sum of |b| must stay below 2^39 mm.
 *   filter   -- Ram-Lak ramp filter along t as a direct convolution over the
 *               row, zero beyond it: q_k = dt sum_n p_n h(k - n), h(0) =
 *               1/(4 dt^2), h(m) = -1/(pi^2 m^2 dt^2) for odd m, 0 otherwise.
 *   back-projection -- x at a voxel centre (x, y) of slice iz =
 *               (pi / n_angles) sum_a q_{iz,a}(t), t = -x sin(a dphi) +
 *               y cos(a dphi), linear interpolation between the lateral bin
 *               centres t0 + (k + 1/2) dt, zero beyond the outer bins.
 * The plan's hull setting does not apply (chords are straight).  Sinograms
 * are device double arrays laid out [iz][a][k] (nz * n_angles * n_t values).
 * Limits: 1 <= n_angles <= 4096, 1 <= n_t <= 4096, nz * n_angles * n_t <
 * 2^31, dt > 0 and t0 finite (PCT_ERR_INVALID_ARG otherwise). */
typedef struct {
    int32_t n_angles; /* angle bins over the full turn                           */
    int32_t n_t;      /* lateral bins                                            */
    double t0, dt;    /* lateral bin k covers [t0 + k dt, t0 + (k+1) dt) (mm)     */
} pct_fbp_geom;

/* Bytes of the FBP workspace (device memory owned by the caller, no upload
 * needed): per bin an int64 sum, a uint32 count and two doubles. */
int pct_fbp_workspace_size(const pct_plan *plan, const pct_fbp_geom *geom, size_t *bytes);

/* Binning: proj (double[nbins]) receives the mean b per bin and count
 * (int32[nbins], may be NULL) the number of protons in it.  b: float[n].
 * Uses the sum and count parts of the FBP workspace. */
int pct_fbp_sinogram(const pct_plan *plan, const pct_fbp_geom *geom, const pct_protons *p, const float *b,
                     double *proj, int32_t *count, void *fbp_ws, size_t fbp_ws_bytes, void *stream);

/* Ramp filter of every row: q (double[nbins]) from proj; the arrays must not
 * overlap. */
int pct_fbp_filter(const pct_plan *plan, const pct_fbp_geom *geom, const double *proj, double *q, void *stream);

/* Back-projection: x (dtype[nvox], overwritten) from the filtered rows q. */
int pct_fbp_backproject(const pct_plan *plan, const pct_fbp_geom *geom, const double *q, void *x, int32_t dtype,
                        void *stream);

/* The three steps: x (dtype[nvox], overwritten) = FBP image of (p, b); the
 * sinograms live in the FBP workspace. */
int pct_fbp(const pct_plan *plan, const pct_fbp_geom *geom, const pct_protons *p, const float *b, void *x,
            int32_t dtype, void *fbp_ws, size_t fbp_ws_bytes, void *stream);

/* ---- diagnostics --------------------------------------------------------- */

/* Kernel timing of the last pct_drop_iterate call made with PCT_DROP_PROFILE:
 * synchronises the recorded events and returns, per kernel kind (index 0: the
 * block kernel, with the commit of the previous block when that is fused into
 * it; 1: the separate commit kernel, none when fused), the summed duration in
 * ms of the sampled launches and their number.  The plan keeps the events; profiling
 * calls on one plan must not overlap. */
int pct_profile_read(pct_plan *plan, double ms[2], int64_t launches[2]);
const char *pct_status_string(int status);
int pct_last_hip_error(void); /* hipError_t of the most recent PCT_ERR_HIP on this thread */

#ifdef __cplusplus
}
#endif
#endif /* PCT_H */
