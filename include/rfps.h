/*
 * rfps.h -- C ABI of the RadiusFPS-G sampling library (librfps.so) for AMD
 * Instinct MI355X (gfx950).
 *
 * The library computes exact farthest point sampling (FPS): the standard FPS
 * loop of Algorithm 1 (Sec. 2.1) with the exactness contract of Sec. 3.1
 * (a fixed start point, one precision throughout, and arg max returning the
 * smallest original index among equal distances).  RadiusFPS (Sec. 3) makes
 * it faster by indexing the cloud with spherical voxels and skipping voxels
 * and points that provably cannot change (Sec. 3.4.2, Sec. 3.4.3); the result
 * is the same sequence plain FPS returns.
 *
 * Distances.  Every distance the library keeps or reports is the FP32
 * squared Euclidean distance ((dx*dx + dy*dy) + dz*dz), dx = fl(p_x - s_x),
 * evaluated without fused multiply-add.  The update is strict: a point's
 * distance changes only when the new value is smaller.
 *
 * Memory.  The caller owns all memory.  Pointers documented as "device" are
 * device (HBM) pointers; "host" pointers are read before the call returns.
 * The library never allocates device memory and keeps no state between
 * calls: everything a call needs lives in the caller's workspace.  A stream
 * argument is a hipStream_t passed as void* (NULL = the default stream); all
 * device work of a call is enqueued on it, in order, and the call returns
 * without waiting for the device unless it says otherwise.
 *
 * Errors.  Argument errors the host can see (sizes, ranges, NULL pointers,
 * a workspace that is too small) are returned at once and nothing is
 * enqueued.  Errors only the device can see (a non-finite coordinate, a
 * cloud that does not fit the on-chip budget, an expired wait) are recorded
 * in the workspace; the sampler then writes -1 to every output index and NaN
 * to every output distance, and rfps_read_status() reports the error.
 */
#ifndef RFPS_H
#define RFPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rfps_status {
    RFPS_OK = 0,
    RFPS_ERR_INVALID_ARG = 1, /* bad size, range or NULL pointer */
    RFPS_ERR_NONFINITE = 2,   /* an input coordinate is NaN or infinite */
    RFPS_ERR_WORKSPACE = 3,   /* workspace NULL, misaligned or too small */
    RFPS_ERR_DEVICE = 4,      /* a HIP runtime call failed */
    RFPS_ERR_UNSUPPORTED = 5, /* no usable gfx950 device, or a launch shape it cannot run */
    RFPS_ERR_CAPACITY = 6,    /* the cloud's share per workgroup exceeds the on-chip budget */
    RFPS_ERR_TIMEOUT = 7,     /* a bounded wait inside a persistent kernel expired */
    RFPS_ERR_INTERNAL = 8,    /* an internal consistency check of a kernel failed */
    RFPS_ERR_SCRATCH_LIMIT = 9 /* input too large for the fixed array of rfps_sample_batched_noalloc */
} rfps_status;

/* rfps_params.flags */
#define RFPS_F_NO_PRUNE 0x01u      /* visit every tile each iteration (no voxel pruning); one-pick sampler */
#define RFPS_F_NO_POINT_SKIP 0x02u /* no coordinate-wise point skip (Sec. 3.4.3) */
#define RFPS_F_TELEMETRY 0x04u     /* count tests, prunes, visits and updates */
#define RFPS_F_TRACE 0x08u         /* time every exchange of workgroup 0 */
#define RFPS_F_SINGLE_PICK 0x10u   /* one selection per exchange (no multi-pick rounds) */
/* Euclidean distances: FPS over the correctly rounded FP32 root of each
 * squared distance, the distance of the update rule of Sec. 3.4.3, instead
 * of the squared value itself.  The two orders differ only where rounding
 * the root merges two distinct squared distances into one value (a tie, then
 * settled by the lower index).  out_d2 then holds Euclidean distances. */
#define RFPS_F_SQRT 0x20u
/* Unfused sampler (rfps_sample only): every selection is its own pair of
 * kernel launches, a selection kernel and a filter/update/resync kernel,
 * ordered by the stream, with the state in device memory between them: the
 * per-iteration-launch variant of the paper's ablation (Sec. 5.4).  Same
 * output; NO_PRUNE, NO_POINT_SKIP and SQRT apply, TELEMETRY and TRACE are
 * not available with it (RFPS_ERR_UNSUPPORTED). */
#define RFPS_F_UNFUSED 0x40u
/* Phase clocks of workgroup 0 of the multi-pick sampler (rfps_sample only),
 * read by rfps_read_telemetry: the instrumented kernel runs with its counters
 * off, so that the clocks see no counting work.  Same output. */
#define RFPS_F_CLOCKS 0x80u

typedef struct rfps_params {
    /* Voxel bins per axis, n_vox of eq. voxel_size (Sec. 3.2); 1..1024.
     * 0 selects the library default for the cloud size. */
    int32_t n_vox;
    /* Largest number of points per tile, 1..64.  A voxel with more points is
     * split into consecutive tiles, each with its own enclosing sphere and
     * its own voxel-level distance.  0 selects 64 (one wavefront). */
    int32_t tile;
    /* Workgroups of the persistent sampler, 1..256 and at most the number of
     * compute units (all must be resident at once); 0 = one per compute unit,
     * or half of them for the multi-pick sampler on clouds below 65,536 points. */
    int32_t groups;
    /* Lookahead depth of the multi-pick sampler: every workgroup proposes
     * this many local candidates per exchange round; 2, 3, 4 or 8 (0 = 2).
     * Output-neutral, like n_vox, tile and groups. */
    int32_t lookahead;
    /* RFPS_F_* bits. */
    uint32_t flags;
    /* Range shells (an extension; output-neutral like every partition):
     * 0 or +inf = one shell, the uniform grid of Sec. 3.2.  A spacing
     * Delta > 0 splits the cloud into shells of width Delta around its
     * bounding-box centre; shell s (distance in [s, s+1) * Delta, the last
     * one open-ended, at most 64) uses cubes of edge (s+1) * L, so sparse
     * far-range points of a spinning sensor share fewer, fuller voxels. */
    float shell_spacing;
} rfps_params;

/* Handle to a voxel index built by rfps_build_index().  Plain data: it
 * records where in the caller's workspace the index lives.  Nothing to free. */
typedef struct rfps_index {
    int32_t n;        /* points */
    int32_t n_vox;    /* resolved voxel bins per axis */
    int32_t tile;     /* resolved tile size */
    int32_t shells;   /* range shells the grid may use (1 = none) */
    void *ws;         /* device workspace holding the index */
    size_t ws_bytes;
} rfps_index;

/* Counters accumulated by a sampling call made with RFPS_F_TELEMETRY. */
typedef struct rfps_telemetry {
    int64_t iters;          /* update rounds after the initial one (m - 2 when m >= 2) */
    int64_t tiles;          /* tiles in the index */
    int64_t tile_tests;     /* sphere tests evaluated */
    int64_t tiles_pruned;   /* tests that skipped the tile */
    int64_t points_visited; /* points in tiles that were not skipped */
    int64_t points_skipped; /* of those, removed by the point skip */
    int64_t points_updated; /* strict decreases of a point's distance */
    int64_t tiles_resynced; /* tiles whose voxel-level distance was recomputed */
    int64_t exchanges;      /* exchange rounds (m - 1 for the one-pick sampler) */
    /* wall-clock ticks workgroup 0 of the multi-pick sampler spent in each
     * phase of its rounds: local lookahead, exchange, merge, apply */
    int64_t ticks_lookahead;
    int64_t ticks_exchange;
    int64_t ticks_merge;
    int64_t ticks_apply;
    int64_t tick_hz;        /* rate of those ticks (filled in by the reader) */
    /* of ticks_exchange, the part spent re-reading slot words that were not
     * yet published at the first pass (waiting for the slowest workgroup) */
    int64_t ticks_wait;
    int64_t reserved;
    /* finer clocks of workgroup 0 (multi-pick sampler, single cloud): the
     * merge's listing (key compaction and any cut of a long list), its
     * ranking pass, its certification walk and its hand-over of the picks;
     * the lookahead's first step (on the true tile state, while the other
     * wavefronts copy it to the private state) and its later steps; the
     * exchange's polling and its forming of the candidate keys */
    int64_t ticks_merge_list;
    int64_t ticks_merge_rank;
    int64_t ticks_merge_walk;
    int64_t ticks_merge_picks;
    int64_t ticks_lookahead_copy;
    int64_t ticks_lookahead_steps;
    int64_t ticks_exchange_poll;
    int64_t ticks_exchange_keys;
    /* per-round merge statistics summed over the rounds: candidates above
     * the largest bound, candidates listed, failed certifications */
    int64_t merge_above;
    int64_t merge_listed;
    int64_t merge_failures;
    /* workgroup 0's own share of the apply phase (its tile loop, without
     * waiting for the other wavefronts) and of the lookahead (choosing each
     * local candidate and its runner-up, without the local updates) */
    int64_t ticks_apply_loop;
    int64_t ticks_lookahead_select;
    /* workgroup 0's first wavefront in the apply phase: clocks of its point
     * updates (tiles some pick reaches), the tile-pick pairs it updated and
     * the tiles it re-keyed */
    int64_t ticks_apply_update;
    int64_t apply_pairs;
    int64_t apply_rekeys;
} rfps_telemetry;

/* Shape of a built index, read back by rfps_read_index_info(). */
typedef struct rfps_index_info {
    int64_t n_voxels;  /* K, active voxels (Sec. 3.2) */
    int64_t n_tiles;   /* tiles after splitting voxels larger than the tile size */
    double pmin[3];    /* bounding-box minimum */
    double voxel_edge; /* L of eq. voxel_size */
} rfps_index_info;

/*
 * Bytes of device workspace that rfps_build_index() and rfps_sample() need
 * for a cloud of n points with these parameters (NULL = defaults).  Returns 0
 * if n < 1 or a parameter is out of range.  Host only; no device work.
 */
size_t rfps_index_workspace_size(int32_t n, const rfps_params *params);

/*
 * Builds the spherical-voxel index of a cloud (Sec. 3.2; the GPU steps of
 * Algorithm 2: voxel mapping, sort by voxel id, gather to structure of
 * arrays, active-voxel compaction), then splits voxels into tiles and
 * computes each tile's enclosing sphere.
 *   xyz      device, float32 [n][3], row-major (x, y, z of point i at 3i..3i+2).
 *            Read only during this call's device work; the index keeps its
 *            own copy, so xyz may be reused once that work has completed.
 *   n        number of points, >= 1.
 *   params   host, may be NULL (defaults).
 *   ws       device workspace, 256-byte aligned, ws_bytes >=
 *            rfps_index_workspace_size(n, params).
 *   out      host; receives the handle.
 * A non-finite coordinate is detected on the device (see rfps_read_status).
 */
rfps_status rfps_build_index(const float *xyz, int32_t n, const rfps_params *params, void *ws,
                             size_t ws_bytes, void *stream, rfps_index *out);

/*
 * Exact FPS of the indexed cloud with spherical-voxel pruning (Sec. 3.3,
 * Sec. 3.4): one persistent kernel runs all m - 1 selections.  By default
 * each exchange between workgroups settles a whole round of selections
 * (certified multi-pick: every workgroup proposes `lookahead` candidates
 * from its own points and all workgroups replay the same exact merge);
 * RFPS_F_SINGLE_PICK exchanges once per selection instead.  Both return the
 * plain FPS sequence bit for bit.
 *   index    host, a handle from rfps_build_index() whose work precedes this
 *            call in stream order.
 *   m        samples, 1 <= m <= n.
 *   start    index of the first sample (the seed s_0), 0 <= start < n.
 *   params   host, may be NULL; only `groups`, `lookahead` and `flags` are read.
 *   out_idx  device, int32 [m]: original indices of the samples in order.
 *   out_d2   device, float32 [m] or NULL: out_d2[0] = +inf; out_d2[j] is the
 *            squared distance of sample j to the nearest earlier sample
 *            (with RFPS_F_SQRT the Euclidean distance, the rounded root).
 * Calls on the same workspace must not overlap (they share its buffers).
 */
rfps_status rfps_sample(const rfps_index *index, int32_t m, int32_t start,
                        const rfps_params *params, int32_t *out_idx, float *out_d2,
                        void *stream);

/*
 * Coordinates of the samples in sample order, out[j] = xyz[idx[j]]: the input
 * of the next stage when a point backbone down-samples in stages (each stage
 * is FPS of the previous stage's samples, start 0).
 *   xyz   device, float32 [n][3] (interleaved x, y, z).
 *   idx   device, int32 [m], e.g. out_idx of rfps_sample; an index outside
 *         [0, n) yields NaN coordinates (a later build reports them).
 *   out   device, float32 [m][3]; must not overlap xyz.
 * Asynchronous on `stream`; host-checked errors return before any work.
 */
rfps_status rfps_gather_xyz(const float *xyz, int32_t n, const int32_t *idx, int32_t m, float *out,
                            void *stream);

/* Waits for the stream, then returns the device-side status recorded in the
 * index workspace by the last build or sampling call (RFPS_OK if none). */
rfps_status rfps_read_status(const rfps_index *index, void *stream);

/* Waits for the stream and copies the index shape into *out (host). */
rfps_status rfps_read_index_info(const rfps_index *index, void *stream, rfps_index_info *out);

/* Waits for the stream and copies the counters of the last sampling call
 * made with RFPS_F_TELEMETRY into *out (host). */
rfps_status rfps_read_telemetry(const rfps_index *index, void *stream, rfps_telemetry *out);

/* Waits for the stream and copies up to `cap` per-iteration timestamps of
 * the last sampling call made with RFPS_F_TRACE into the host array `out`:
 * one pair per exchange (per selection for the one-pick sampler, per round
 * for the multi-pick sampler): out[2k] is the time workgroup 0 published
 * its candidates for exchange k, out[2k+1] the time it knew the outcome, in
 * ticks of the device wall clock; for the multi-pick sampler the top 16 bits
 * of out[2k+1] hold the number of selections the round settled (mask them
 * off before using the time).  *ticks_per_s receives the clock's rate.
 * Returns the number of pairs. */
/*
 * Latency floor of the sampler's exchange (measurement only): `groups`
 * workgroups (0 = one per compute unit, at most 256) run `rounds` exchanges
 * of `words` (1..64) epoch-tagged 64-bit words each per workgroup, with
 * nothing else in a round, through the same agent-scope stores, loads and
 * polling as the multi-pick sampler (which publishes 6 * lookahead + 2
 * words).  Uses the index's exchange board and trace buffer as scratch (the
 * next sampling call clears the board; the last trace is overwritten).
 * Waits for the stream.  *us_per_round receives the wall-clock time per
 * exchange of workgroup 0.  RFPS_ERR_TIMEOUT if a bounded wait expired.
 */
rfps_status rfps_probe_exchange(const rfps_index *index, int32_t groups, int32_t words, int32_t rounds,
                                void *stream, double *us_per_round);

int32_t rfps_read_trace(const rfps_index *index, void *stream, uint64_t *out, int32_t cap,
                        double *ticks_per_s);

/*
 * Plain FPS without any index (the comparison kernels):
 *   variant 0: persistent, every workgroup keeps its share of the points and
 *              of D in registers, one exchange per selection;
 *   variant 1: one workgroup streams the whole cloud from device memory every
 *              selection (the conventional GPU FPS kernel).
 * Arguments as above; ws is device workspace of
 * rfps_fps_plain_workspace_size(n, variant) bytes.  groups applies to
 * variant 0 (0 = one per compute unit).
 */
size_t rfps_fps_plain_workspace_size(int32_t n, int32_t variant);
rfps_status rfps_fps_plain(const float *xyz, int32_t n, int32_t m, int32_t start, int32_t variant,
                           int32_t groups, void *ws, size_t ws_bytes, int32_t *out_idx,
                           float *out_d2, void *stream);

/* Waits for the stream, then returns the device-side status recorded in a
 * plain-FPS workspace by the last rfps_fps_plain() call on it. */
rfps_status rfps_read_plain_status(const void *ws, size_t ws_bytes, void *stream);

/*
 * Batches of clouds.  The exact FPS of Algorithm 1 (Sec. 2.1, with the
 * Sec. 3.1 tie rule) runs independently on every cloud of a batch; one call
 * builds one spherical-voxel index over all clouds (Sec. 3.2, every cloud on
 * its own grid) and samples all of them in one persistent launch.  Teams of
 * `groups` workgroups, each team on one XCD, take the clouds from a queue
 * ordered by decreasing N_c * m_c.  Output-neutral like the single-cloud
 * parameters: the selections of every cloud equal plain FPS on that cloud.
 *   xyz       device, float32 [n][3]: the clouds one after the other.
 *   n         total points, 1 <= n <= 2^26.
 *   offsets   device, int32 [batch + 1]: cloud c is points offsets[c] ..
 *             offsets[c+1]-1; offsets[0] = 0, offsets[batch] = n, and every
 *             cloud has at least one point.
 *   m         device, int32 [batch]: selections of cloud c, 1 <= m[c] <= N_c.
 *   starts    device, int32 [batch] or NULL: local index of the first sample
 *             of cloud c, 0 <= starts[c] < N_c (NULL: all 0).
 *   batch     clouds, 1 <= batch <= min(4096, n).
 *   m_total   sum of m[c]: the length of the outputs (checked on the device).
 *   params    host, may be NULL.  n_vox: 0 = per-cloud default bins, else
 *             the same bins for every cloud; tile as for rfps_build_index;
 *             groups: workgroups per cloud (a divisor of the compute units of
 *             one XCD, at least 2; 0 = all of them); lookahead 2, 3, 4 or 8 (0 =
 *             2).  RFPS_F_NO_PRUNE, RFPS_F_SINGLE_PICK and RFPS_F_TRACE are
 *             not available here (RFPS_ERR_UNSUPPORTED).
 *   ws        device workspace of rfps_batched_workspace_size() bytes,
 *             256-byte aligned; calls on one workspace must not overlap.
 *   out_idx   device, int32 [m_total]: the selections of cloud c at
 *             m[0] + .. + m[c-1] onwards, as indices local to the cloud.
 *   out_d2    device, float32 [m_total] or NULL: distances as for
 *             rfps_sample, per cloud (each cloud's first entry is +inf).
 * The call allocates nothing and never waits for the device, so it may be
 * captured into a HIP graph (under capture the persistent kernel is an
 * ordinary launch after a residency check).  Device-side errors (offsets,
 * m, starts or m_total inconsistent, non-finite input, capacity) are
 * recorded in the workspace; all outputs then become -1 / NaN.
 */
size_t rfps_batched_workspace_size(int32_t n, int32_t batch, const rfps_params *params);
rfps_status rfps_sample_batched(const float *xyz, int32_t n, const int32_t *offsets,
                                const int32_t *m, const int32_t *starts, int32_t batch,
                                int32_t m_total, const rfps_params *params, void *ws,
                                size_t ws_bytes, int32_t *out_idx, float *out_d2, void *stream);

/*
 * rfps_sample_batched without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc).  Same method, arguments (minus ws and
 * ws_bytes), outputs and device-side error behaviour (outputs -1 / NaN) as
 * rfps_sample_batched.  The workspace is a fixed array inside the library,
 * rfps_noalloc_scratch_bytes() = 128 MiB per device, created when the
 * library's device code is loaded on that device and held until the process
 * ends; the call allocates nothing (no hipMalloc, no allocating library call).
 *   Limit: rfps_batched_workspace_size(n, batch, params) must not exceed that
 *   size (RFPS_ERR_SCRATCH_LIMIT otherwise, with nothing enqueued); about
 *   1.7 M points in 32 clouds.
 *   Sharing: every call on one device uses that device's one array, and the
 *   array keeps the last call's contents (each call clears what must start at
 *   zero itself).  Calls in one stream order are safe; calls that overlap on
 *   one GPU (two streams or threads at once) race and give undefined
 *   results.  The device-side status word stays in the array and has no
 *   reader: check the outputs for -1 / NaN.
 */
size_t rfps_noalloc_scratch_bytes(void);
rfps_status rfps_sample_batched_noalloc(const float *xyz, int32_t n, const int32_t *offsets,
                                        const int32_t *m, const int32_t *starts, int32_t batch,
                                        int32_t m_total, const rfps_params *params, int32_t *out_idx,
                                        float *out_d2, void *stream);

/* Waits for the stream and returns the device-side status the last batched
 * call recorded in ws (RFPS_OK if none). */
rfps_status rfps_batched_read_status(const void *ws, size_t ws_bytes, void *stream);

/* Waits for the stream and copies the counters of the last batched call made
 * with RFPS_F_TELEMETRY (summed over all clouds; the phase clocks stay 0). */
rfps_status rfps_batched_read_telemetry(const void *ws, size_t ws_bytes, void *stream,
                                        rfps_telemetry *out);

/*
 * Autotuner for batched calls: times rfps_sample_batched on this batch for
 * every combination of groups (per_xcd, per_xcd/2, .. down to 4), lookahead
 * (2, 3, 4, 8) and tile (32, 64) that `base` leaves at 0 (non-zero fields of
 * base are kept), `reps` timed runs each after one untimed run, and returns
 * the fastest by median in *best (host) and its median in *best_ms (host,
 * may be NULL).  Shapes the device cannot hold (RFPS_ERR_CAPACITY,
 * RFPS_ERR_UNSUPPORTED) are skipped; every other candidate must reproduce
 * the first one's selections exactly (else RFPS_ERR_INTERNAL).  On return
 * the outputs hold the result of the chosen configuration.  Synchronous:
 * it waits for the device and is not for use under graph capture.
 */
rfps_status rfps_autotune_batched(const float *xyz, int32_t n, const int32_t *offsets,
                                  const int32_t *m, const int32_t *starts, int32_t batch,
                                  int32_t m_total, const rfps_params *base, int32_t reps,
                                  void *ws, size_t ws_bytes, int32_t *out_idx, float *out_d2,
                                  void *stream, rfps_params *best, float *best_ms);

/* Static description of a status code. */
/*
 * CPU RadiusFPS (Sec. 3, the paper's CPU method) on the host cores: the
 * same plain FPS sequence as the GPU samplers and the same readings (grid,
 * enclosing spheres, FP-safe skip threshold, tie-break), run by a team of
 * threads that each own every T-th tile and meet at one barrier per
 * selection.
 *   xyz      host, float32 [n][3]; 1 <= n <= 2^26.
 *   m        samples, 1 <= m <= n; start as for rfps_sample.
 *   params   host, may be NULL: n_vox (0 = half of rfps_default_n_vox(n),
 *            at least 8: larger voxels suit the host's cores), tile
 *            (0 = 64) and flags (RFPS_F_SQRT; RFPS_F_NO_POINT_SKIP is
 *            accepted and changes nothing) are read.
 *   threads  team size; 0 = OMP_NUM_THREADS if set, else the CPUs the
 *            process may run on.  Each member spins at the barrier, so the
 *            team should not exceed the cores available.
 *   out_idx  host, int32 [m]; out_d2 host, float32 [m] or NULL (as for
 *            rfps_sample).
 * Synchronous; allocates host memory for its index and state (about 60
 * bytes per point) and frees it before returning.  Non-finite input returns
 * RFPS_ERR_NONFINITE, and host memory or threads that cannot be obtained
 * RFPS_ERR_INTERNAL; both leave the outputs -1 / NaN.
 */
rfps_status rfps_cpu_sample(const float *xyz, int32_t n, int32_t m, int32_t start,
                            const rfps_params *params, int32_t threads, int32_t *out_idx,
                            float *out_d2);

const char *rfps_status_str(rfps_status s);

/* Default voxel bins per axis for a cloud of n points. */
int32_t rfps_default_n_vox(int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* RFPS_H */
