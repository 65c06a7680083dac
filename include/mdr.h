/*
 * mdr.h -- C ABI of the MI355X (gfx950) bitplane refactor / progressive retrieve
 * library, after HP-MDR (arXiv 2505.00227).
 *
 * Plain C: opaque handles, plain pointers and sizes, no C++ exceptions cross
 * this boundary.  Device pointers are HIP device memory on the context's
 * device; `stream` arguments are hipStream_t values passed as void* (NULL =
 * the device's default stream).  Every function returns an mdr_status; on any
 * error an output handle is set to NULL, retriever state is left unchanged,
 * and mdr_last_error() returns a message for the calling thread.
 *
 * What the operations compute (paper sections):
 *   refactor  = per level: alignment to the level's largest exponent and
 *               sign/magnitude fixed point (Sec. 3, Alg. 1 step 1), bitplanes
 *               most significant first (Sec. 3, Alg. 1 loop), an exact per-plane
 *               L-infinity error table (MDR's error estimate, Sec. 2.2), then
 *               hybrid lossless coding of merged plane groups (Sec. 4, Alg. 2:
 *               Huffman / run-length / direct copy with placeholders).
 *   retrieve  = progressive, incremental reconstruction to an error bound
 *               (Sec. 1 and 5: fetch just enough precision segments), the
 *               inverse of the above.
 *   QoI       = retrieval until the V_total = vx^2+vy^2+vz^2 error estimate
 *               meets a tolerance (Sec. 5.2, Alg. 3 with the MAPE estimator).
 */
#ifndef MDR_H
#define MDR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDR_MAX_PLANES 64

typedef enum {
    MDR_OK = 0,
    MDR_ERR_INVALID_ARG = 1,    /* bad argument, or NaN / Inf in the input       */
    MDR_ERR_UNSUPPORTED = 2,    /* valid request this build does not handle      */
    MDR_ERR_OUT_OF_MEMORY = 3,  /* device or host allocation failed              */
    MDR_ERR_HIP = 4,            /* a HIP runtime call failed                     */
    MDR_ERR_CORRUPT_STREAM = 5, /* serialized data failed a header/size/CRC check */
    MDR_ERR_BUSY = 6            /* resource limit reached; retry later            */
} mdr_status;

typedef enum { MDR_F32 = 0, MDR_F64 = 1 } mdr_dtype;

/* lossless method of one stream (Sec. 4; placeholders are Alg. 2's empty slots) */
typedef enum { MDR_DC = 0, MDR_RLE = 1, MDR_HUF = 2, MDR_PLACEHOLDER = 3 } mdr_method;

/* MDR_REL: tolerance x (max - min over every coefficient of the variable) */
/* MDR_L2: absolute bound on the L2 norm of the variable's coefficient error,
 * sqrt(sum over levels of E2[k]) <= tol; mdr_retrieve only, after
 * mdr_l2_table. */
typedef enum { MDR_ABS = 0, MDR_REL = 1, MDR_L2 = 2 } mdr_bound;

/* Codec parameters of Alg. 2.  Every field is recorded in the serialized form. */
typedef struct {
    uint32_t group_planes; /* m: planes per lossless group (default 4; >= 1, capped at nplanes) */
    uint32_t t_cr_milli;   /* T_cr x 1000: ratio threshold (default 2000)                       */
    uint64_t t_s_bytes;    /* T_s: groups of at most this many bytes are copied (default 4096)   */
    uint32_t huf_chunk;    /* byte symbols per Huffman chunk (default 256; 256, 512 .. 4096)    */
    uint32_t huf_lmax;     /* longest Huffman code (default 12; 8..12)                           */
    int32_t force_method;  /* -1: Alg. 2 decides (default); MDR_DC/RLE/HUF: used for every unit  */
} mdr_codec_params;

/* One coefficient level: n values of the variable's dtype in device memory.
 * Borrowed: must stay valid until the work queued on the call's stream ends. */
typedef struct {
    const void* data;
    uint64_t n;
} mdr_level_view;

typedef struct {
    double tol_abs;          /* absolute tolerance this call planned for                    */
    double bound;            /* L-inf bound reached: sum over levels of E_l[k_l]            */
    uint64_t bytes_fetched;  /* stream bytes this call decoded (new groups only)            */
    uint64_t bytes_held;     /* stream bytes held by the retriever after the call           */
    uint32_t groups_fetched; /* lossless units this call decoded                           */
    int32_t met;             /* 1 if bound <= tol_abs, 0 if every plane is held and it is not */
} mdr_retrieve_info;

typedef struct mdr_context mdr_context;
typedef struct mdr_refactored mdr_refactored;
typedef struct mdr_retriever mdr_retriever;

/* ---------------------------------------------------------------- library */
const char* mdr_version(void);
/* Message of the last failed call on this thread ("" if none).  Valid until the
 * thread's next mdr_* call. */
const char* mdr_last_error(void);
/* Fills the defaults listed in mdr_codec_params. */
mdr_status mdr_codec_params_default(mdr_codec_params* out);

/* ---------------------------------------------------------------- context */
/* A context binds one HIP device and owns reusable device workspaces.
 * Calls on one context must not run concurrently from several host threads. */
mdr_status mdr_context_create(int hip_device, mdr_context** out);
void mdr_context_destroy(mdr_context* ctx);

/* Per-stage device timing.  When enabled, every kernel launch of the library is
 * bracketed by HIP events on the stream it runs on; mdr_context_timing waits for
 * them and returns, per stage, the summed kernel milliseconds and launch counts
 * (arrays of MDR_STAGE_COUNT entries; reset != 0 clears the totals afterwards).
 * Timing adds a few microseconds per launch; off by default. */
typedef enum {
    MDR_STAGE_STATS = 0,       /* level statistics (alignment exponent)          */
    MDR_STAGE_ENCODE = 1,      /* bitplane encoder + error table + group stats    */
    MDR_STAGE_SELECT = 2,      /* Alg. 2 selection and Huffman codebooks          */
    MDR_STAGE_LOSSLESS = 3,    /* Huffman + run-length encoding, sizes, offsets   */
    MDR_STAGE_ASSEMBLE = 4,    /* metadata (tables, sizes, methods) to the host   */
    MDR_STAGE_HUF_DECODE = 5,
    MDR_STAGE_RLE_DECODE = 6,
    MDR_STAGE_RECONSTRUCT = 7, /* bitplane decoder + reconstruction               */
    MDR_STAGE_COUNT = 8
} mdr_stage;
mdr_status mdr_context_set_timing(mdr_context* ctx, int enable);
mdr_status mdr_context_timing(mdr_context* ctx, double* ms, uint64_t* launches, int reset);

/* Launch shape of the refactor pass (the autotuner's knobs; results do not
 * depend on them, bit for bit):
 *   enc_target_wg   encoder workgroups a pass aims for (tiles of 256 blocks are
 *                   split evenly among them); 64..65536, default 2304;
 *   stats_wg_values values per statistics workgroup (at most 256 workgroups
 *                   per level); 1024..2^24, default 65536.
 * Zero leaves a knob unchanged.  `graphs` (0/1, -1 = unchanged): whether
 * mdr_refactor_batch captures and replays HIP graphs (default 1). */
mdr_status mdr_context_set_launch(mdr_context* ctx, uint32_t enc_target_wg, uint32_t stats_wg_values,
                                  int graphs);

/* Lanes that decode one Huffman chunk in a retrieval (Sec. 4.2's chunked
 * codes; results do not depend on it, bit for bit).  1: one thread a chunk,
 * a serial walk of its codes through a table of up to three symbols a
 * lookup (the launch for many chunks).  4, 8, 16, 32 or 64: the chunk's
 * bits are cut into that many ranges, decoded at once and brought into step
 * (a prefix code resynchronises), which shortens a launch with few chunks;
 * raised to chunk/64 where a stream's chunk needs it.  0 (the default):
 * chosen per launch, one lane from 3 x 2^24 symbols on, else 16 symbols a
 * lane (capped at 64 lanes).  Other values: MDR_ERR_INVALID_ARG. */
mdr_status mdr_context_set_decode_lanes(mdr_context* ctx, uint32_t lanes);

/* ---- Launch-shape autotuner (the batched pass's block and tile shapes) ----
 * A launch shape is the three knobs of the refactor pass: enc_target_wg and
 * stats_wg_values (above) and select_threads, the workgroup size of the
 * Alg. 2 selection kernel (256, 512 or 1024, or 0: chosen per pass, 256 when
 * the pass selects at least 1024 units (levels x groups), 512 below; default
 * 0).  No knob changes a result, bit for bit; only time.
 *
 * The context keeps a tuning table keyed by (dtype, nplanes, group size,
 * floor(log2(values in the pass)), floor(log2(levels in the pass))); a pass
 * whose key has an entry runs at that entry's shape, any other pass at the
 * context's default shape (mdr_context_set_launch / _set_select_threads).
 *
 * mdr_autotune_refactor: times refactor passes over the given variables (the
 * arguments of mdr_refactor_batch; the results are discarded) at the default
 * shape and at candidate shapes, by coordinate descent (encoder workgroups,
 * then statistics workgroup values, then selection threads; `reps` passes per
 * shape, the fastest counted; HIP events on `stream`), and records the fastest
 * in the table.  With force = 0 and an entry already present for the key, it
 * times nothing and reports that entry (candidates = 0).  Waits for `stream`.
 * mdr_tune_save / mdr_tune_load: write / read the table as JSON (one entry per
 * line); load merges into the table (a missing file is MDR_ERR_INVALID_ARG,
 * a malformed one MDR_ERR_CORRUPT_STREAM).  mdr_context_create loads the file
 * named by the environment variable MDR_TUNE_CACHE when it exists, and with
 * MDR_AUTOTUNE=1 a pass whose key has no entry is tuned first (then the file,
 * if named, is rewritten). */
typedef struct {
    uint32_t enc_target_wg;
    uint32_t stats_wg_values;
    uint32_t select_threads;
} mdr_launch_shape;
typedef struct {
    mdr_launch_shape best;     /* the recorded shape */
    mdr_launch_shape dflt;     /* the context's default shape */
    double best_ms;            /* fastest pass at `best` (0 when taken from the table) */
    double default_ms;         /* fastest pass at the default shape (0 likewise) */
    uint32_t candidates;       /* shapes timed, 0 = taken from the table */
    uint32_t value_bucket;     /* floor(log2(values in the pass)) */
    uint32_t level_bucket;     /* floor(log2(levels in the pass)) */
} mdr_tune_result;
mdr_status mdr_context_set_select_threads(mdr_context* ctx, uint32_t threads);
mdr_status mdr_autotune_refactor(mdr_context* ctx, const mdr_level_view* const* vars, const uint32_t* nlevels,
                                 uint32_t nvars, mdr_dtype dtype, uint32_t nplanes,
                                 const mdr_codec_params* params, void* stream, uint32_t reps, int force,
                                 mdr_tune_result* out);
mdr_status mdr_tune_save(const mdr_context* ctx, const char* path);
mdr_status mdr_tune_load(mdr_context* ctx, const char* path);
/* number of table entries, and entry i's key and shape (for inspection) */
mdr_status mdr_tune_entries(const mdr_context* ctx, uint32_t* count);
mdr_status mdr_tune_entry(const mdr_context* ctx, uint32_t i, uint32_t key[5], mdr_launch_shape* shape);

/* ---------------------------------------------------------------- refactor */
/*
 * Refactor one variable given as nlevels coefficient levels (coarsest first).
 * Per level (Sec. 3, Alg. 1; Sec. 4, Alg. 2):
 *   e      = largest frexp exponent of its nonzero values (|x| < 2^e; 0 if all zero);
 *   mag    = floor(|x| * 2^(nplanes - e)), sign = sign bit;
 *   planes = plane p holds bit nplanes-1-p of every value; value i is bit i of the
 *            plane's little-endian byte string, padded to a whole W-bit word
 *            (W = 32 for f32, 64 for f64);
 *   E[k]   = max |x - xhat^(k)| after k planes, k = 0..nplanes (exact);
 *   units  = the sign plane, then groups of m planes, each coded DC/RLE/HUF.
 * nplanes: 1..32 for f32, 1..64 for f64 (else MDR_ERR_UNSUPPORTED).
 * NaN or Inf anywhere -> MDR_ERR_INVALID_ARG.  A level may be empty (n = 0).
 * `params` may be NULL (defaults).  Work is queued on `stream`; the call returns
 * after the small metadata (sizes, methods, error tables) is on the host.
 * Stream sizes are decided on the device: payload memory is reserved for the
 * largest stream each unit's method could produce (about S / T_cr under Alg. 2).
 * The result owns its device streams; free with mdr_refactored_destroy.
 */
mdr_status mdr_refactor(mdr_context* ctx, const mdr_level_view* levels, uint32_t nlevels,
                        mdr_dtype dtype, uint32_t nplanes, const mdr_codec_params* params,
                        void* stream, mdr_refactored** out);
void mdr_refactored_destroy(mdr_refactored* r);

/*
 * Refactor nvars variables at once (same dtype, nplanes and params; variable v
 * has nlevels[v] levels at vars[v]).  Results equal nvars separate
 * mdr_refactor calls, bit for bit.  The whole batch is one pass: one launch per
 * stage over every level of every variable, with stream sizes decided on the
 * device and one metadata copy at the end.  With graphs on (the default), the
 * pass is captured as a HIP graph the first time a batch of this shape (level
 * sizes, input alignment, params) is seen, and replayed afterwards; at most 8
 * shapes are kept per context.  outs[v] receives variable v's handle (all NULL
 * on error); the handles share device arenas, released with the last of them.
 */
mdr_status mdr_refactor_batch(mdr_context* ctx, const mdr_level_view* const* vars,
                              const uint32_t* nlevels, uint32_t nvars, mdr_dtype dtype,
                              uint32_t nplanes, const mdr_codec_params* params, void* stream,
                              mdr_refactored** outs);

mdr_status mdr_refactored_shape(const mdr_refactored* r, uint32_t* nlevels, mdr_dtype* dtype,
                                uint32_t* nplanes, mdr_codec_params* params);
/* Level metadata: e, n, min, max (a zero of either sign reads +0.0), and
 * error_table[0..nplanes] (exact values of the dtype, widened to double).
 * Any output pointer may be NULL. */
mdr_status mdr_refactored_info(const mdr_refactored* r, uint32_t level, int32_t* e, uint64_t* n,
                               double* vmin, double* vmax, double* error_table);
/* One stream of a level: stream -1 = sign plane, 0..nplanes-1 = magnitude plane p
 * (a group's payload sits at its leading plane; the group's other planes are
 * MDR_PLACEHOLDER with 0 bytes).  *dev_ptr points into memory owned by r. */
mdr_status mdr_refactored_stream(const mdr_refactored* r, uint32_t level, int32_t stream,
                                 const void** dev_ptr, uint64_t* bytes, mdr_method* method);

/* Container (Sec. 5.1 serialization): little-endian header, per-level records
 * with error tables, stream table with CRC-32 per payload, payloads.
 * cap = 0 (host may be NULL) -> *used = required size, MDR_OK. */
mdr_status mdr_serialize(const mdr_refactored* r, void* host, uint64_t cap, uint64_t* used);
/* Validates magic, version, sizes and every CRC (MDR_ERR_CORRUPT_STREAM on any
 * mismatch), then uploads the streams to the context's device. */
mdr_status mdr_deserialize(mdr_context* ctx, const void* host, uint64_t bytes,
                           mdr_refactored** out);

/* ---------------------------------------------------------------- retrieve */
/* A retriever holds, for one refactored variable, the planes fetched so far
 * (per level) and the decoded form of its compressed groups.  `r` must outlive it. */
mdr_status mdr_retriever_create(mdr_context* ctx, const mdr_refactored* r, mdr_retriever** out);
void mdr_retriever_destroy(mdr_retriever* rt);

/*
 * Progressive, incremental retrieval: plan (greedy, from the planes already held)
 * the planes per level whose bound sum_l E_l[k_l] <= tol (absolute, or relative
 * to the variable's value range), decode only groups not held yet, and write
 * every level's reconstruction x = (-1)^sign * (top k_l bits of mag) * 2^(e - nplanes)
 * to level_out[l] (device, n_l values of the dtype; k_l = 0 writes +0.0).
 * The result equals a fresh retrieval to the same planes, bit for bit.
 * A tolerance below the all-planes bound returns MDR_OK with info->met = 0.
 * Queued on `stream`; `info` (may be NULL) is filled on return.
 */
mdr_status mdr_retrieve(mdr_retriever* rt, mdr_bound kind, double tol, void* const* level_out,
                        void* stream, mdr_retrieve_info* info);
/* Same, with the planes per level given explicitly (each k_l is rounded up to a
 * whole group and may not go below what is already held). */
mdr_status mdr_retrieve_planes(mdr_retriever* rt, const uint32_t* k, void* const* level_out,
                               void* stream, mdr_retrieve_info* info);
/* Retrieval for n retrievers at once (each at most once): retriever i plans to
 * tols[i] (kind as in mdr_retrieve) and writes level_out[i][l].  Results equal n
 * separate mdr_retrieve calls, bit for bit; the work is one Huffman-decode
 * launch for every group that enters a plan and one reconstruction launch per
 * dtype for every level of every variable.  infos (n entries) may be NULL.
 * On error no retriever changes. */
mdr_status mdr_retrieve_batch(mdr_retriever* const* rts, uint32_t n, mdr_bound kind,
                              const double* tols, void* const* const* level_out, void* stream,
                              mdr_retrieve_info* infos);
/* Planes currently held per level (nlevels entries). */
mdr_status mdr_retriever_planes(const mdr_retriever* rt, uint32_t* k);

typedef struct {
    double tau_abs;          /* absolute V_total tolerance the call worked to                  */
    double tau_est;          /* final estimate tau' (every point's V_total error is <= it)     */
    double eps[3];           /* final L-inf bounds of vx, vy, vz                               */
    uint64_t bytes_fetched;  /* stream bytes decoded by this call, all three variables          */
    uint32_t iterations;     /* estimate / re-plan rounds of Alg. 3                             */
    int32_t met;             /* 1 if tau_est <= tau_abs, 0 if every plane is held and it is not */
} mdr_qoi_info;

/*
 * Retrieval with error control on V_total = vx^2 + vy^2 + vz^2 (Sec. 5.2, Alg. 3,
 * with the MAPE estimator).  The three retrievers must describe variables with the
 * same dtype and the same number of values per level (points correspond one to
 * one; recomposition is the identity).  Starting from the planes each holds:
 *   eps_c = (tau / Q_max) * range_c, Q_max = sum_c max(|min_c|, |max_c|)^2, and each
 *   variable is planned to eps_c; then repeat: reconstruct, eps_c = bound of the
 *   planes held, tau' = (1 + 2^-40) * max_p sum_c eps_c (2|v_c(p)| + eps_c) (double,
 *   x, y, z order); stop if tau' <= tau or every plane is held; else p = tau'/tau:
 *   if p > mape_c, re-plan each variable to eps_c / p; if that adds nothing (or
 *   p <= mape_c) fetch one more merged group per variable (minimal augmentation).
 * kind: MDR_ABS (tau as given) or MDR_REL (tau x Q_max).  mape_c <= 0 means 10.
 * Reconstructions are left in out_x / out_y / out_z (device, per level).
 * On error the retrievers keep every group decoded so far (their state stays valid).
 */
mdr_status mdr_retrieve_qoi_vtotal(mdr_retriever* vx, mdr_retriever* vy, mdr_retriever* vz,
                                   mdr_bound kind, double tau, double mape_c,
                                   void* const* out_x, void* const* out_y, void* const* out_z,
                                   void* stream, mdr_qoi_info* info);

/*
 * The three next-bound estimators of Sec. 5.2 for the loop above:
 *   MDR_QOI_MAPE  the loop above (minimal augmentation with proportional estimation);
 *   MDR_QOI_MA    minimal augmentation only: one more merged group per variable
 *                 per round (MAPE that never takes the proportional step);
 *   MDR_QOI_CP    the CPU-porting estimator: at the point with the largest estimate
 *                 (the first in level-concatenated order among equal ones, found on
 *                 the device), every bound is multiplied by cp_decay until that
 *                 point's estimate, evaluated from its current values exactly as
 *                 tau' is, is within tau (at most 2200 times); each variable is then
 *                 re-planned to its bound.
 * For all three, a round whose bounds add no group fetches one more merged group
 * per variable, as above.
 */
typedef enum { MDR_QOI_MAPE = 0, MDR_QOI_MA = 1, MDR_QOI_CP = 2 } mdr_qoi_estimator;
typedef struct {
    int32_t estimator;  /* mdr_qoi_estimator                                        */
    uint32_t pad;
    double mape_c;      /* MAPE threshold c; <= 0 means 10                            */
    double cp_decay;    /* CP factor per step, in (0, 1); <= 0 means 1/2              */
} mdr_qoi_params;
/* mdr_retrieve_qoi_vtotal with a chosen estimator (params NULL: MAPE, c = 10).
 * An estimator outside the enum, or cp_decay >= 1, is MDR_ERR_INVALID_ARG. */
mdr_status mdr_retrieve_qoi_vtotal_with(mdr_retriever* vx, mdr_retriever* vy, mdr_retriever* vz,
                                        mdr_bound kind, double tau, const mdr_qoi_params* params,
                                        void* const* out_x, void* const* out_y, void* const* out_z,
                                        void* stream, mdr_qoi_info* info);

/*
 * Further QoI families (Sec. 5.2 controls errors of derived quantities; the
 * families below are this library's reading of that error estimation).  The
 * loop, the estimators and the retriever requirements are those of
 * mdr_retrieve_qoi_vtotal_with, over nvars retrievers rts[] (distinct, same
 * dtype and points per level) writing outs[c][l]; per family, at every point,
 * from the reconstruction vhat_c and the planes' bounds eps_c:
 *   MDR_QOI_SUMSQ      S = sum_c v_c^2, nvars 1..3 (3: V_total):
 *                      score D = sum_c eps_c (2|vhat_c| + eps_c); tau' = max D;
 *                      scale Q_max = sum_c A_c^2 (A_c = max(|min_c|, |max_c|));
 *                      initial eps_c = (tau / Q_max) range_c.
 *   MDR_QOI_MAGNITUDE  M = sqrt(S), nvars 1..3: |M - Mhat| <= D / Mhat and
 *                      <= sqrt(sum_c eps_c^2); score D^2 / Shat (+inf at
 *                      Shat = 0), tau' = sqrt(min(sum_c eps_c^2, max score));
 *                      scale sqrt(Q_max); initial eps_c = tau / sqrt(nvars).
 *   MDR_QOI_PRODUCT    P = v_0 v_1, nvars 2: score (|vhat_0| eps_1 +
 *                      |vhat_1| eps_0) + eps_0 eps_1; tau' = max score; scale
 *                      A_0 A_1; initial eps_0 = tau / (2 A_1), eps_1 = tau / (2 A_0).
 * tau' is inflated by (1 + 2^-40) (rounding cover); MDR_REL multiplies tau by
 * the scale.  info->eps holds the first nvars bounds.  Bad family, variable
 * count or estimator: MDR_ERR_INVALID_ARG.
 */
typedef enum { MDR_QOI_SUMSQ = 0, MDR_QOI_MAGNITUDE = 1, MDR_QOI_PRODUCT = 2 } mdr_qoi_kind;
mdr_status mdr_retrieve_qoi(mdr_qoi_kind family, mdr_retriever* const* rts, uint32_t nvars, mdr_bound kind,
                            double tau, const mdr_qoi_params* params, void* const* const* outs, void* stream,
                            mdr_qoi_info* info);

/* ---------------------------------------------------------------- chunked pipeline */
/*
 * A field held in host memory as nchunks chunks, each an independent
 * sub-domain of nlevels levels (sizes level_sizes[], coarsest first; chunk c's
 * values at host + c * chunk_values, levels concatenated).  Refactor: the H2D
 * copy of chunk c+1, the refactor of chunk c and the D2H copy of chunk c-1's
 * streams overlap on three streams (overlap = 0: one stage at a time, the
 * unpipelined reference); the streams stay in the pipeline's pinned host
 * memory.  Retrieve: the H2D copy of chunk c+1's streams, the decode and
 * reconstruction of chunk c and the D2H copy of chunk c-1's values overlap
 * likewise; every chunk is planned to the same absolute tolerance (MDR_REL:
 * tol x the whole field's value range).  Each chunk's result equals
 * mdr_refactor / mdr_retrieve of that chunk alone, bit for bit.  host_values /
 * host_out should be pinned (hipHostMalloc) for the copies to overlap.
 */
typedef struct mdr_pipeline mdr_pipeline;
typedef struct {
    double wall_ms;                     /* whole call, host clock                               */
    double h2d_ms, compute_ms, d2h_ms;  /* summed device time of each stream's work (events)   */
    uint64_t h2d_bytes, d2h_bytes;      /* bytes copied each way                                 */
    uint64_t stream_bytes;              /* refactor: stream bytes made; retrieve: bytes decoded */
} mdr_pipeline_info;

mdr_status mdr_pipeline_create(mdr_context* ctx, uint32_t nchunks, const uint64_t* level_sizes,
                               uint32_t nlevels, mdr_dtype dtype, uint32_t nplanes,
                               const mdr_codec_params* params, mdr_pipeline** out);
mdr_status mdr_pipeline_refactor(mdr_pipeline* p, const void* host_values, int overlap,
                                 mdr_pipeline_info* info);
mdr_status mdr_pipeline_retrieve(mdr_pipeline* p, mdr_bound kind, double tol, void* host_out,
                                 int overlap, mdr_pipeline_info* info);
/* A device copy of one refactored chunk (for inspection or serialization). */
mdr_status mdr_pipeline_chunk(const mdr_pipeline* p, uint32_t chunk, mdr_context* ctx,
                              mdr_refactored** out);
void mdr_pipeline_destroy(mdr_pipeline* p);

/* ---------------------------------------------------------------- serving */
/*
 * A retrieval server keeps refactored fields resident in HBM and serves
 * requests from an engine thread with continuous batching: every engine step
 * advances every admitted request by one round (a field request finishes in one
 * round; a V_total request takes the rounds of mdr_retrieve_qoi_vtotal), with
 * one batched decode, one batched reconstruction and one batched estimate for
 * all of them on the server's own stream.  A request is admitted when one of
 * max_slots slots and the HBM for its outputs (within hbm_budget) are free; the
 * others wait in arrival order.  Decoded groups are cached per field and shared
 * by every request on it, so planes fetched once are reused.  A request's
 * result depends only on its own tolerance and starting planes: it is the same,
 * bit for bit, alone or in any mix, and equal to mdr_retrieve /
 * mdr_retrieve_qoi_vtotal from the same planes.  The server uses a context of
 * its own on ctx's device; fields must outlive the server.  Each output
 * component is one device block (one field's reconstruction); released blocks
 * are kept for the next request and reused, so the device memory the server
 * holds for outputs never exceeds hbm_budget and steady serving allocates none.
 */
typedef struct mdr_server mdr_server;

typedef enum { MDR_REQ_FIELD = 0, MDR_REQ_QOI_VTOTAL = 1 } mdr_request_kind;

typedef struct {
    int32_t kind;        /* MDR_REQ_FIELD: field[0]; MDR_REQ_QOI_VTOTAL: vx, vy, vz = field[0..2] */
    uint32_t field[3];
    int32_t bound;       /* MDR_ABS, or MDR_REL (field: x value range; QoI: x Q_max)              */
    double tol;          /* L-inf tolerance (field) or V_total tolerance (QoI)                    */
    double mape_c;       /* QoI: MAPE threshold (<= 0 means 10)                                   */
    uint64_t parent;     /* 0, or the ticket of an earlier request of the same kind and fields:   */
                         /* start from the planes it ended with (an incremental refinement)       */
    uint64_t tag;        /* echoed in the completion                                              */
} mdr_request;

typedef struct {
    uint64_t ticket, tag;
    int32_t status;          /* mdr_status of the request                                          */
    int32_t met;             /* bound <= tol_abs                                                   */
    double tol_abs;          /* absolute tolerance worked to                                       */
    double bound;            /* field: L-inf bound of the planes used; QoI: the estimate tau'      */
    uint64_t bytes_fetched;  /* stream bytes of groups beyond the starting planes                  */
    uint32_t iterations;     /* engine rounds taken                                               */
    uint32_t pad;
    double t_submit_ms, t_start_ms, t_done_ms;  /* server clock (ms since creation)             */
} mdr_completion;

typedef struct {
    uint32_t pending, active, completed_unreleased, pad;
    uint64_t steps;          /* engine steps so far                                                */
    uint64_t step_requests;  /* sum over steps of the requests advanced (batching depth)           */
    uint64_t hbm_in_use, hbm_budget;
    uint64_t hbm_held;       /* output blocks allocated (in use, or kept for reuse): <= hbm_budget */
} mdr_server_info;

mdr_status mdr_server_create(mdr_context* ctx, uint64_t hbm_budget, uint32_t max_slots, mdr_server** out);
/* Registers a refactored field (while no request is queued); ids count from 0. */
mdr_status mdr_server_add_field(mdr_server* s, const mdr_refactored* r, uint32_t* field_id);
/* Queues a request and returns at once.  Rejected at once (no ticket): bad
 * fields, mismatched QoI fields, outputs larger than the budget, unknown parent. */
mdr_status mdr_server_submit(mdr_server* s, const mdr_request* req, uint64_t* ticket);
/* Copies up to cap completions (oldest first) and returns at once. */
mdr_status mdr_server_poll(mdr_server* s, mdr_completion* out, uint32_t cap, uint32_t* n);
/* Device output of a completed request: component comp (0 for a field request;
 * 0..2 = x, y, z for QoI), level `level`, n values of the field's dtype.  Valid
 * until mdr_server_release(ticket). */
mdr_status mdr_server_output(mdr_server* s, uint64_t ticket, uint32_t comp, uint32_t level, void** dev_ptr,
                             uint64_t* n);
/* Returns a completed request's outputs to the budget. */
mdr_status mdr_server_release(mdr_server* s, uint64_t ticket);
mdr_status mdr_server_stats(mdr_server* s, mdr_server_info* info);
/* Stops the engine (queued requests are dropped) and frees everything. */
void mdr_server_destroy(mdr_server* s);

/*
 * Encoder-design ablation (Sec. 3; the encoding experiments of Sec. 6): n 32-bit
 * words into 32 bitplanes (plane p = bit 31 - p) and back, with no alignment,
 * error table or lossless stage, by each parallelisation the paper compares:
 *   MDR_ABL_LOCALITY   a thread per block of 32 contiguous values (the layout
 *                      the refactor path uses);
 *   MDR_ABL_BALLOT     a value per lane, one wavefront vote per bit;
 *   MDR_ABL_SHIFT      a value per lane, a five-round OR tree per bit;
 *   MDR_ABL_BUTTERFLY  a value per lane, the 32x32 transpose across 32 lanes in
 *                      five exchange rounds;
 *   MDR_ABL_REGBLOCK   the register block: lane l of each 2048-value region holds
 *                      its values l, l+64, ..., l+1984 (coalesced loads).
 * Layouts: plane-major, mdr_ablation_plane_words(design, n) words per plane.
 * Every design but the register block: word j holds bit t of value 32j + t.
 * Register block: word 64r + l holds, at bit k, value 2048r + l + 64k.  Values
 * past n count as 0.  in / planes / out: device memory, 16-byte aligned, owned
 * by the caller; work is enqueued on `stream`.  Unknown design, NULL or
 * misaligned pointers: MDR_ERR_INVALID_ARG.
 */
typedef enum {
    MDR_ABL_LOCALITY = 0,
    MDR_ABL_BALLOT = 1,
    MDR_ABL_SHIFT = 2,
    MDR_ABL_BUTTERFLY = 3,
    MDR_ABL_REGBLOCK = 4
} mdr_ablation_design;
uint64_t mdr_ablation_plane_words(int32_t design, uint64_t n);
mdr_status mdr_ablation_encode(int32_t design, const uint32_t* in, uint64_t n, uint32_t* planes, void* stream);
mdr_status mdr_ablation_decode(int32_t design, const uint32_t* planes, uint64_t n, uint32_t* out, void* stream);

/* ---- Squared-L2 per-plane table (the MDR L2 option) -----------------------
 * The paper controls L-infinity error throughout; MDR also offers an L2 error
 * table, which this adds beside the exact L-infinity one.  E2[k] =
 * sum_i (x_i - xhat_i^(k))^2 over a level, k = 0..nplanes, where xhat^(k) is
 * the k-plane reconstruction; residuals are exact, squares rounded once, sums
 * in fp64 in a fixed order (the same on every run).
 * mdr_l2_table: computes the tables of every level of `r` from the values it
 * was refactored from (`levels`, nlevels and each n as given to mdr_refactor;
 * device memory, borrowed), keeps them in `r`, and waits for `stream`.
 * Mismatched counts or sizes, NULL, misaligned or non-device data:
 * MDR_ERR_INVALID_ARG; so are values whose largest |x| in some level differs
 * from the refactored level's (other data than `r` was refactored from: no
 * table is kept).  A deserialized object has no table until this runs.
 * mdr_refactored_l2: copies level `level`'s table (nplanes + 1 doubles) to
 * host memory; MDR_ERR_INVALID_ARG if there is none.
 * With the tables, mdr_retrieve(kind = MDR_L2, tol) plans the fewest groups
 * (same greedy planner) with sum_l E2_l[k_l] <= tol^2; info->bound is then
 * the L2 bound sqrt(sum_l E2_l[k_l]). */
mdr_status mdr_l2_table(mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, void* stream);
mdr_status mdr_refactored_l2(const mdr_refactored* r, uint32_t level, double* E2);

/* mdr_l2_table_noalloc: mdr_l2_table for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, tables and errors, computed by the same kernels (bit-identical
 * tables); the partial sums and tables live in a fixed scratch array of the
 * library (574,464 bytes per device, resolved once per device by
 * mdr_context_create and held until the process ends) instead of pool memory,
 * and no hipMalloc, hipFree or allocating library routine is called.
 * nlevels above 64: MDR_ERR_UNSUPPORTED.  Every call on one device shares that
 * scratch, so calls that overlap on one device (other host threads, or other
 * streams before this call's wait returns) race and must be serialized by the
 * caller. */
mdr_status mdr_l2_table_noalloc(mdr_refactored* r, const mdr_level_view* levels, uint32_t nlevels, void* stream);

/* ---- Multilevel decomposition (the coefficient levels of Sec. 2/3) ---------
 * The method's input is the coefficient levels of a multilevel decomposition
 * that the paper takes from earlier work without spelling it out.  Reading
 * used here: hierarchical multilinear interpolation (MGARD's interpolation
 * step, no L2-projection correction).  The field is row-major n0 x n1 x n2
 * (n2 fastest).  Step j (j = 0 finest) works on the stride h = 2^j grid; each
 * of its nodes not on the stride-2h grid gets c = u - P, where P refines the
 * stride-2h values along n2, then n1, then n0: (a + b) * 0.5 of the two
 * neighbours on the axis, or the left neighbour alone past the last coarse
 * node of a line.  Arithmetic is in the field's type, one rounding per
 * operation.  Level 0 holds the raw values of the stride-2^nsteps grid; level
 * l (1..nsteps) holds the nodes of step nsteps - l in the row-major order of
 * their grid.  P is a convex combination, so after recomposition the field's
 * max error is at most the sum of the levels' max coefficient errors (plus
 * rounding): a tolerance met on the levels is met on the field.
 *
 * mdr_level_sizes: host only; sizes[nsteps + 1] = values per level.
 * mdr_decompose: field (n0*n1*n2 values) -> coeffs, the levels concatenated
 *   coarsest first (level l at offset sizes[0] + ... + sizes[l-1]).
 * mdr_recompose: the inverse; every value of `field` is written.
 * Both: device memory owned by the caller, aligned to the value size, not
 * overlapping; work is enqueued on `stream` (one launch to decompose,
 * nsteps + 1 to recompose).  nsteps <= 30 (steps past the grid's extent give
 * empty levels); n0, n1 < 65536 and n2 < 2^31, else MDR_ERR_UNSUPPORTED;
 * NULL, misaligned or overlapping buffers, a buffer that is not inside one
 * device allocation of at least n0*n1*n2 values, a bad dtype or nsteps:
 * MDR_ERR_INVALID_ARG.  An empty grid is a no-op. */
mdr_status mdr_level_sizes(uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps, uint64_t* sizes);
mdr_status mdr_decompose(mdr_dtype dtype, const void* field, uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps,
                         void* coeffs, void* stream);
mdr_status mdr_recompose(mdr_dtype dtype, const void* coeffs, uint64_t n0, uint64_t n1, uint64_t n2, uint32_t nsteps,
                         void* field, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MDR_H */
