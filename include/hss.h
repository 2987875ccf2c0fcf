/*
 * hss.h -- Histogram Sort with Sampling on one MI355X (gfx950).
 *
 * C ABI of libhss.so.  The method is the one of Harsh, Kale and Solomonik,
 * "Histogram Sort with Sampling" (SPAA'19): the p processors of the paper are
 * p contiguous segments of one device buffer, segment s holding the input
 * positions [floor(s N / p), floor((s+1) N / p)).
 *
 * Conventions shared by every entry point
 *   - Device pointers are caller-owned and must stay valid until the work
 *     enqueued on `stream` has completed.  Inputs are never modified.
 *     Outputs must not overlap inputs; every device pointer must be 16-byte
 *     aligned.  Violations return HSS_ERR_INVALID_ARG before any work is
 *     enqueued.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued on `stream`.  The splitter rounds are queued k at
 *     a time (k of section 4.2) and read a few counter words back to the
 *     host after them (and after every further round, if one is needed),
 *     and hss_partition / hss_sort read the device consistency word once
 *     more at the end, so both return after their work on `stream` has
 *     completed.  Every segment sort also reads back how many of its
 *     sub-buckets overflow on-chip memory, so hss_local_sort returns after
 *     its work has completed too.
 *   - Keys are unsigned integers (32 or 64 bit) compared as unsigned.  Equal
 *     keys are ordered by (source segment, position in the segment), the
 *     implicit tags of section 6.1, which makes every result equal to what a
 *     stable sort of the input would give.
 *   - A payload, when given, is one uint64_t per key moved with its key.
 *   - No C++ exception crosses this interface.  On failure the status is
 *     returned and hss_last_error() holds a message for the calling thread.
 */
#ifndef HSS_H
#define HSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The last enumerator gives the type the range of a 32-bit int, so that any
 * int a C caller passes is a value of the type (out-of-range values are
 * rejected with HSS_ERR_INVALID_ARG). */
typedef enum { HSS_U32 = 0, HSS_U64 = 1, HSS_KEY_TYPE_INT_RANGE_ = 0x7FFFFFFF } hss_key_type;

typedef enum {
    HSS_OK = 0,
    HSS_ERR_INVALID_ARG = -1,    /* bad sizes, null or misaligned pointers, overlap */
    HSS_ERR_UNSUPPORTED = -2,    /* a valid request the library does not handle     */
    HSS_ERR_OUT_OF_MEMORY = -3,  /* device allocation failed                        */
    HSS_ERR_DEVICE = -4,         /* HIP error or a failed device-side consistency check */
    HSS_ERR_NOT_CONVERGED = -5,  /* tuning.max_rounds reached with splitters unsettled */
    HSS_ERR_CANCELLED = -6       /* a server request taken out of the queue         */
} hss_status;

typedef struct hss_plan_s* hss_plan_t;

/* Optional knobs; zero-initialise for the defaults. */
typedef struct {
    uint32_t max_rounds;        /* 0: no cap.  The schedule reaches rate 1 after a
                                   bounded number of rounds, which settles every
                                   splitter, so the default always converges.    */
    uint32_t k_override;        /* 0: k = max(1, ceil(ln(2 ln p / eps))) (section 4.2) */
    uint32_t force_full_sample; /* 1: every key is a probe in round 1 (one round) */
    uint32_t trace_level;       /* 0: per-round counts only; 1: also probes, ranks
                                   and splitter state per round (host copies);
                                   2: also every round's local histograms      */
    uint32_t lsd_only;          /* 1: sort segments and buckets by plain 8-bit LSD
                                   passes instead of the MSD pass + on-chip finish
                                   (same results; for comparison)               */
    uint32_t probes_per_round;  /* c > 0: a fixed budget of c p probes per round
                                   (the implementation of section 6 and the
                                   theorem with O(p) samples per round): each key
                                   of the round's domain gamma is a probe with
                                   probability min(1, c p / |gamma|), in place of
                                   the rate schedule; single plans only          */
    uint32_t plain_launches;    /* 1: launch every round kernel; 0: the rounds
                                   queued before the first read-back run from a
                                   HIP graph captured once per plan (captured
                                   again when the probe buffers grow)           */
    uint32_t autotune;          /* 1: the first call tries the launch knobs of
                                   hss_knobs on its own input, one knob at a
                                   time, and moves off the current knobs only
                                   for a setting more than 2% faster (the
                                   outputs do not depend on the knobs)          */
    uint32_t workspace_limit_mib; /* 0: no limit.  Otherwise the most device
                                   memory, in MiB, the plan (for a batch: the
                                   instances of each key type) may take:
                                   a plan whose workspace (its tables, two key
                                   buffers and the first probe buffers) would
                                   exceed it fails with HSS_ERR_OUT_OF_MEMORY
                                   before any device call, and so does a later
                                   growth of its probe buffers past it        */
    uint32_t pick_sampler;      /* 1 (with probes_per_round = c): draw the probes
                                   as the implementation of section 6 does:
                                   every segment picks ceil(c N / |gamma|)
                                   uniform positions of its whole sorted input
                                   (with replacement; Philox counter (pick,
                                   segment, round, 1)) and keeps those inside
                                   the splitter intervals, each position once;
                                   when that reaches the largest segment every
                                   key of the intervals is taken.  The round
                                   trace reports the pick count as the round's
                                   threshold.  Single plans only              */
    uint32_t reserved[1];       /* must be zero */
} hss_tuning;

/* Launch knobs of a plan (hss_plan_knobs); none changes any output. */
typedef struct {
    uint32_t small_sort_cap;    /* keys sorted on chip per job of the local
                                   sort: 2048 or 4096                           */
    uint32_t sample_workgroups; /* grid of the sampler                          */
    uint32_t pair_rank_from;    /* first round whose ranks are searched per
                                   (probe, segment) inside the probe's interval
                                   slice; earlier rounds by segment chunks     */
    uint32_t pair_rank_workgroups; /* grid of that search                       */
    uint32_t tuned;             /* 1 once the autotuner has run                 */
} hss_knobs;

/*
 * hss_plan -- validate (N, p, eps, key type) and prepare a plan.
 *   n            number of keys N, 1 <= p <= N (section 2: N/p keys per processor)
 *   p            number of segments ("processors") and of output buckets
 *   eps          balance tolerance, 0 < eps < 1: every splitter rank lies in
 *                [N i/p - tol, N i/p + tol] with tol = floor(N eps / (2p))
 *                (target range, section 2), so no bucket exceeds
 *                ceil(N/p) + 2 tol <= N (1 + eps) / p + 1 keys
 *   kt           HSS_U32 or HSS_U64 keys
 *   with_payload 1 if calls will pass a uint64_t payload per key
 *   tuning       NULL for defaults
 * The plan owns a device workspace of hss_workspace_bytes(plan) bytes,
 * allocated on the current device.  A plan may be reused for any number of
 * calls; calls on one plan must not overlap in time.
 * N must be below 2^32 (HSS_ERR_UNSUPPORTED otherwise): tags, counts and
 * piece offsets are 32-bit words.  That is 16 GiB of u32 or 32 GiB of u64
 * keys on one device; 64-bit tags would double the count matrix, the
 * per-cell tables and the probe arrays for inputs that one device does not
 * hold with its workspace anyway.
 */
hss_status hss_plan(hss_plan_t* out, uint64_t n, uint32_t p, double eps, hss_key_type kt,
                    int with_payload, const hss_tuning* tuning);

/*
 * hss_plan_buckets -- as hss_plan, but the p segments are split into
 * 1 <= q <= p buckets: one stage of HSS with several stages (section 5.3),
 * where q groups of processors take one bucket each.  The splitters are
 * i = 1..q-1 with ideal ranks N i/q; the tolerance floor(N eps / (2q)), the
 * final sampling ratio 2 ln q / eps and the rate q s_j / N of section 4.2
 * count buckets, the histograms still run over the p segments.  With such
 * a plan hss_partition and hss_sort write q buckets and q+1 offsets, the
 * trace calls report q-1 splitters and a (q+1) x p piece matrix.  q = p is
 * hss_plan.  Errors as hss_plan; q outside 1..p is HSS_ERR_INVALID_ARG.
 */
hss_status hss_plan_buckets(hss_plan_t* out, uint64_t n, uint32_t p, uint32_t q, double eps,
                            hss_key_type kt, int with_payload, const hss_tuning* tuning);

/* Release a plan and its device memory (synchronises the device). NULL is ok. */
void hss_plan_destroy(hss_plan_t plan);

/* Bytes of device memory held by the plan. */
size_t hss_workspace_bytes(hss_plan_t plan);

/*
 * hss_partition -- the partition of HSS (section 4.2.2 steps 1-5, then the
 * data exchange of section 3.1 step 3 done as one bucketed scatter).
 *   seed          selects the Philox4x32-10 stream of the sampling rounds
 *   d_keys_in     N keys (uint32_t or uint64_t per the plan)
 *   d_vals_in     N payload words, or NULL for a keys-only plan
 *   d_keys_out    N keys: bucket b = 0..p-1 occupies [chi(b), chi(b+1)) and holds
 *                 the keys of global rank chi(b)..chi(b+1)-1, as pieces in
 *                 ascending source segment, each piece in local sorted order
 *   d_vals_out    N payload words moved with the keys (NULL iff d_vals_in NULL)
 *   d_offsets     p+1 uint64_t: chi(0) = 0, chi(1..p-1) = splitter ranks, chi(p) = N
 */
hss_status hss_partition(hss_plan_t plan, uint64_t seed, const void* d_keys_in,
                         const uint64_t* d_vals_in, void* d_keys_out, uint64_t* d_vals_out,
                         uint64_t* d_offsets, void* stream);

/*
 * hss_sort -- hss_partition followed by a stable sort of every bucket
 * (the local merge after the exchange, section 5): the output is the stable
 * sort of the input by key.  Same arguments and offsets as hss_partition.
 */
hss_status hss_sort(hss_plan_t plan, uint64_t seed, const void* d_keys_in,
                    const uint64_t* d_vals_in, void* d_keys_out, uint64_t* d_vals_out,
                    uint64_t* d_offsets, void* stream);

/*
 * hss_partition_static -- hss_partition for callers that cannot allocate
 * device memory: code that runs under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  There is no plan: the call takes the
 * shape (n, p, eps, key type; a payload iff d_vals_in is given) and its
 * workspace is one fixed device array of the library,
 * HSS_STATIC_SCRATCH_MIB MiB per device, reserved when the library's code
 * is loaded on that device and held until the process ends.  The call
 * allocates no device or pinned host memory (its read-backs go through a
 * static host buffer); it launches on `stream` only (no side stream, no
 * graph) and returns after its work has completed, like hss_partition.
 * Outputs and offsets are exactly those of hss_partition on a plan of the
 * same shape for the same seed and input.
 *   Limits: n <= HSS_STATIC_MAX_KEYS and p <= HSS_STATIC_MAX_BUCKETS, and
 *   the shape's workspace (hss_partition_static_bytes) must fit the array;
 *   otherwise HSS_ERR_UNSUPPORTED with a message.  A round whose sample
 *   overruns the probe buffers that fit the array returns
 *   HSS_ERR_OUT_OF_MEMORY.
 *   Every call on a device uses that device's one array and leaves its last
 *   contents there (the kernels clear what they need).  The library runs such
 *   calls one at a time (a mutex), and each returns after its work has
 *   completed, so two calls never use the array at once; a caller that
 *   issued device work touching the array by other means would race with it.
 */
#define HSS_STATIC_SCRATCH_MIB 96u
#define HSS_STATIC_MAX_KEYS (1u << 20)
#define HSS_STATIC_MAX_BUCKETS 256u

hss_status hss_partition_static(uint64_t n, uint32_t p, double eps, hss_key_type kt, uint64_t seed,
                                const void* d_keys_in, const uint64_t* d_vals_in, void* d_keys_out,
                                uint64_t* d_vals_out, uint64_t* d_offsets, void* stream);

/* Bytes of the fixed array a hss_partition_static call of this shape takes,
 * and the array's size; computed on the host (no device call).  Returns the
 * status hss_partition_static would give for the shape. */
hss_status hss_partition_static_bytes(uint64_t n, uint32_t p, double eps, hss_key_type kt,
                                      int with_payload, size_t* bytes, size_t* capacity);

/*
 * hss_partition_ws -- hss_partition with the caller's device workspace: a
 * call on no plan that takes every device word it needs from d_workspace
 * (256-byte aligned, workspace_bytes long, not overlapping the inputs or
 * outputs) and allocates no device memory.  Section 2's problem, as
 * hss_partition: the same outputs for the same seed.  The workspace must hold
 * at least hss_partition_workspace_bytes for the shape (else
 * HSS_ERR_INVALID_ARG before any device call); a call whose probe rounds
 * overrun the 4x headroom that size includes fails with
 * HSS_ERR_OUT_OF_MEMORY, its outputs unwritten.  The workspace's contents
 * are scratch between calls; calls sharing one workspace must not overlap in
 * time.  Returns after the work on `stream` has completed.
 */
hss_status hss_partition_ws(uint64_t n, uint32_t p, double eps, hss_key_type kt, uint64_t seed,
                            const void* d_keys_in, const uint64_t* d_vals_in, void* d_keys_out,
                            uint64_t* d_vals_out, uint64_t* d_offsets, void* d_workspace,
                            size_t workspace_bytes, void* stream);

/* Bytes of workspace a hss_partition_ws call of this shape needs (*bytes = 0
 * and the shape's error for a shape hss_partition would refuse). */
hss_status hss_partition_workspace_bytes(uint64_t n, uint32_t p, double eps, hss_key_type kt,
                                         int with_payload, size_t* bytes);

/*
 * hss_local_sort -- only the first phase (section 6, local sort): every
 * segment sorted stably by key, payload moved with its key.  The output
 * position of an element is its tag g.
 */
hss_status hss_local_sort(hss_plan_t plan, const void* d_keys_in, const uint64_t* d_vals_in,
                          void* d_keys_out, uint64_t* d_vals_out, void* stream);

/*
 * hss_get_constants -- the plan's round constants (section 4.2).
 *   tol         floor(N eps / (2p))
 *   k           rounds of the rate schedule s_j = a^(j/k)
 *   a           2 ln p / eps (= s_k)
 *   thresh[j-1] for j = 1..max_j: a key of the round-j domain is a probe when
 *               its Philox word is below thresh; all[j-1] = 1 when every key
 *               is taken (p s_j / N >= 1).  Either array may be NULL.
 */
hss_status hss_get_constants(hss_plan_t plan, uint64_t* tol, uint32_t* k, double* a,
                             uint32_t max_j, uint32_t* thresh, uint32_t* all);

/* Trace of the last hss_partition / hss_sort call on the plan (host data). */
uint32_t hss_trace_rounds(hss_plan_t plan);

/* Round j (0-based): domain size |gamma_{j}| sampled from, probe count m,
 * acceptance threshold and the all-keys flag. */
hss_status hss_trace_round_info(hss_plan_t plan, uint32_t j, uint64_t* domain, uint64_t* m,
                                uint32_t* thresh, uint32_t* all);

/* Round j probes in sorted order: keys, tags g and global ranks R (m each;
 * any pointer may be NULL).  Needs trace_level >= 1. */
hss_status hss_trace_round_probes(hss_plan_t plan, uint32_t j, uint64_t* keys, uint64_t* tags,
                                  uint64_t* ranks);

/* Round j local histograms (section 4.2.2 step 2): counts[e p + s] = c_s(e),
 * the number of keys of segment s that precede probe e (in sorted probe
 * order) in the order (key, segment, index) of section 6.1; m x p words.
 * Their sum over s is the probe's rank R.  Needs trace_level >= 2. */
hss_status hss_trace_round_counts(hss_plan_t plan, uint32_t j, uint32_t* counts);

/* Splitter state after round j, p-1 entries each: rank of the bounding probe
 * below / above N i/p (UINT64_MAX for none or settled), settled flag, chi
 * (0 while unsettled).  Needs trace_level >= 1. */
hss_status hss_trace_round_state(hss_plan_t plan, uint32_t j, uint64_t* lo_rank,
                                 uint64_t* hi_rank, uint8_t* settled, uint64_t* chi);

/* Final splitters: chi (p+1), key and tag of S(i) (p+1; entries 0 and p are
 * unused), and the piece matrix ((p+1) x p, row b = per-segment count of
 * keys preceding S(b)).  Any pointer may be NULL. */
hss_status hss_trace_splitters(hss_plan_t plan, uint64_t* chi, uint64_t* s_key, uint64_t* s_tag,
                               uint64_t* pieces);

/*
 * Measurement.  hss_profile(plan, 1) makes later calls on the plan bracket
 * every launch of a kernel family with HIP events recorded on the call's
 * stream; hss_profile_read waits for those events and returns, for one
 * family, the summed milliseconds, the number of launches and the
 * algorithmic bytes the launches move (keys, payload and tables read plus
 * written).  Families:
 *   0 radix count   1 radix scan   2 radix scatter
 *   3 splitter rounds (the whole phase, host read-backs included; bytes 0)
 *   4 exchange offsets   5 exchange copy   6 on-chip sub-bucket sort
 * hss_profile(plan, 0) stops timing; hss_profile_reset zeroes the totals.
 */
hss_status hss_profile(hss_plan_t plan, int enable);
hss_status hss_profile_reset(hss_plan_t plan);
hss_status hss_profile_read(hss_plan_t plan, uint32_t family, double* ms, uint64_t* launches,
                            uint64_t* bytes);

/*
 * Batches: many independent instances (each its own N, p, eps, key type and
 * seed) partitioned together.  Every phase -- local sort, splitter rounds,
 * exchange -- processes all instances of one key type in the same launches,
 * so the per-launch and per-round costs are paid once per batch instead of
 * once per instance.  Each instance's result is exactly what hss_partition
 * of a plan with the same (N, p, eps, key type, payload) returns for its
 * seed and input.
 */
typedef struct hss_batch_s* hss_batch_t;

typedef struct {
    uint64_t n;                 /* keys N of the instance, 1 <= p <= N      */
    uint32_t p;                 /* segments and buckets                     */
    hss_key_type key_type;      /* HSS_U32 or HSS_U64                       */
    double eps;                 /* 0 < eps < 1, as in hss_plan              */
} hss_instance_shape;

typedef struct {
    uint64_t seed;              /* Philox stream of the instance's rounds   */
    const void* keys_in;        /* N keys                                   */
    const uint64_t* vals_in;    /* N payload words, or NULL without payload */
    void* keys_out;             /* N keys in buckets (each bucket sorted    */
                                /* for HSS_OP_SORT)                         */
    uint64_t* vals_out;         /* N payload words, or NULL                 */
    uint64_t* offsets;          /* p+1 words: chi                           */
} hss_instance_io;

/*
 * hss_batch_plan -- validate `count` instance shapes and prepare a batch:
 * one workspace per key type present, sized for the sum of the instances.
 * The sum of N per key type must stay below 2^32.  tuning: NULL, or knobs
 * as for hss_plan except lsd_only and trace_level, which must be zero
 * (HSS_ERR_UNSUPPORTED otherwise); a probe budget (probes_per_round = c)
 * applies to every instance, each with its own rate c q / |gamma| from its
 * own domain.  Errors name the failing instance.
 */
hss_status hss_batch_plan(hss_batch_t* out, const hss_instance_shape* shapes, uint32_t count,
                          int with_payload, const hss_tuning* tuning);

/* Release a batch and its device memory (synchronises the device). NULL is ok. */
void hss_batch_destroy(hss_batch_t batch);

/* Bytes of device memory held by the batch. */
size_t hss_batch_workspace_bytes(hss_batch_t batch);

/*
 * hss_batch_partition -- hss_partition of every instance: io[i] holds the
 * buffers of shape i (same conventions and checks as hss_partition, per
 * instance).  Returns after the work on `stream` has completed.
 */
hss_status hss_batch_partition(hss_batch_t batch, const hss_instance_io* io, void* stream);

/* Measurement of a batch, summed over its key types; families as for
 * hss_profile_read. */
hss_status hss_batch_profile(hss_batch_t batch, int enable);
hss_status hss_batch_profile_reset(hss_batch_t batch);
hss_status hss_batch_profile_read(hss_batch_t batch, uint32_t family, double* ms,
                                  uint64_t* launches, uint64_t* bytes);

/*
 * Server: requests of any shape arriving over time, each an hss_partition or
 * an hss_sort of its own input (the served workload: independent sorts
 * submitted by clients), with continuous batching.  Worker threads of the
 * server, each on a stream of its own, take the requests queued when they
 * become free -- in submission order, of one operation, key type and payload
 * choice, within the batch limits; a sort request runs alone (its bucket sort
 * is per plan) -- and run them as one batch; requests that arrive while other
 * batches are on the GPU start on a free worker as soon as the HBM budget
 * admits them, so their work overlaps on the device.  A request is admitted
 * when its footprint (inputs, outputs and its share of the workspace)
 * fits the budget left by the batches running (a request above the whole
 * budget runs when nothing else does).  Device memory comes from a cache of
 * blocks kept between batches (no allocation once the cache covers the
 * load).  Every request's outputs equal those of hss_partition (or hss_sort)
 * of a plan with its (N, p, eps, key type, payload) for its seed and input.
 */
typedef enum {
    HSS_OP_PARTITION = 0,       /* hss_partition: buckets of locally sorted pieces */
    HSS_OP_SORT = 1,            /* hss_sort: every bucket sorted                   */
    HSS_OP_INT_RANGE_ = 0x7FFFFFFF
} hss_op;

typedef struct hss_server_s* hss_server_t;

typedef struct {
    uint64_t n;                 /* keys N, 1 <= p <= N                      */
    uint32_t p;                 /* buckets                                  */
    hss_key_type key_type;      /* HSS_U32 or HSS_U64                       */
    double eps;                 /* 0 < eps < 1                              */
    uint64_t seed;              /* Philox stream of the request's rounds    */
    const void* keys_in;        /* N keys on the device, fully written when */
                                /* submitted (the server's streams do not   */
                                /* wait on the writer's)                    */
    const uint64_t* vals_in;    /* N payload words, or NULL                 */
    void* keys_out;             /* N keys, bucket order as hss_partition    */
    uint64_t* vals_out;         /* N payload words iff vals_in              */
    uint64_t* offsets;          /* p+1 words: chi                           */
    hss_op op;                  /* HSS_OP_PARTITION (0) or HSS_OP_SORT      */
} hss_request;

typedef struct {
    uint64_t max_batch_keys;    /* keys per batch (0: 2^30; below 2^32); a  */
                                /* single larger request still runs, alone  */
    uint32_t max_batch_requests;/* requests per batch (0: 1024)             */
    uint32_t workers;           /* batches on the GPU at once (0: 2)        */
    uint64_t hbm_budget;        /* bytes of admitted requests' footprints   */
                                /* at once (0: 64 GiB)                      */
    uint32_t batch_wait_us;     /* a free worker whose queue head is a      */
                                /* partition request with no other of its   */
                                /* class queued waits up to this long after */
                                /* the head's submission for one (0: never; */
                                /* batching for latency)                    */
} hss_server_config;

/* hss_server_create -- start a server on the current device; cfg NULL: the
 * defaults above. */
hss_status hss_server_create(hss_server_t* out, const hss_server_config* cfg);

/* Bytes a request counts against the budget: its inputs and outputs and the
 * workspace of its keys in a batch. */
uint64_t hss_server_footprint(const hss_request* req);

/* Finish every submitted request, stop the worker and release the server's
 * memory.  NULL is ok. */
void hss_server_destroy(hss_server_t server);

/*
 * hss_server_submit -- queue a request; *ticket names it.  The buffers stay
 * owned by the caller and must remain valid until the request is done.
 * Argument errors (shape, pointers, alignment, overlap) are returned here and
 * nothing is queued; device errors come back as the request's result.
 */
hss_status hss_server_submit(hss_server_t server, const hss_request* req, uint64_t* ticket);

/*
 * hss_server_poll -- *done = 1 when the request has finished (its outputs are
 * written and visible to any stream); then *result is its status and
 * t_submit / t_done its submission and completion times on
 * hss_server_clock, and the ticket is retired.  *done = 0: still queued or
 * running.  Unknown tickets: HSS_ERR_INVALID_ARG.  Output pointers may be NULL.
 */
hss_status hss_server_poll(hss_server_t server, uint64_t ticket, int* done, hss_status* result,
                           double* t_submit, double* t_done);

/*
 * hss_server_cancel -- take a queued request out of the queue: *cancelled = 1
 * and the request is done with result HSS_ERR_CANCELLED, its outputs
 * untouched (poll or wait still retires the ticket).  A request that a worker
 * has already taken (running or done) is left to finish: *cancelled = 0.
 * Unknown tickets: HSS_ERR_INVALID_ARG.  cancelled may be NULL.
 */
hss_status hss_server_cancel(hss_server_t server, uint64_t ticket, int* cancelled);

/* hss_server_wait -- as hss_server_poll, blocking until the request is done. */
hss_status hss_server_wait(hss_server_t server, uint64_t ticket, hss_status* result,
                           double* t_submit, double* t_done);

/* Seconds on the server's monotonic clock (the clock of t_submit, t_done). */
double hss_server_clock(void);

/* Since creation: batches run, requests finished and their keys, the most
 * batches on the GPU at once and the most budget bytes admitted at once. */
hss_status hss_server_stats(hss_server_t server, uint64_t* batches, uint64_t* requests,
                            uint64_t* keys, uint32_t* max_concurrent, uint64_t* max_admitted);

/* Device bytes the server's block cache holds now (blocks of running
 * batches and idle ones kept for reuse) and the most it has held.  Idle
 * blocks are freed, largest first, whenever the total would exceed the HBM
 * budget, so the total stays within it unless the running batches alone
 * need more. */
hss_status hss_server_memory(hss_server_t server, uint64_t* held, uint64_t* max_held);

/* The launch knobs a plan (or, for a batch, its instances of one key type)
 * runs with: the defaults, or what the autotuner chose on the first call. */
hss_status hss_plan_knobs(hss_plan_t plan, hss_knobs* out);
/* Set a plan's launch knobs (small_sort_cap 2048 or 4096, grids in [1, 65536],
 * pair_rank_from >= 1; `tuned` is kept as given).  HSS_ERR_INVALID_ARG on
 * other values. */
hss_status hss_plan_set_knobs(hss_plan_t plan, const hss_knobs* knobs);
hss_status hss_batch_knobs(hss_batch_t batch, hss_key_type kt, hss_knobs* out);

/*
 * ------------------------------------------------------------ two stages --
 * HSS with two stages (section 5.3): the p processors form r groups of p/r.
 * Stage 1 splits the N keys into r buckets, one per group (tolerance eps1,
 * as hss_plan_buckets with q = r), and moves every bucket to its group.
 * The group's keys are then dealt out evenly to its p/r processors in the
 * order the exchange wrote them, and stage 2 runs HSS inside every group on
 * its own (tolerance eps2, Philox seed `seed + 1 + g` for group g), all
 * groups in the same launches.  Final bucket g p/r + i is bucket i of group
 * g, so every bucket holds at most about N (1 + eps1)(1 + eps2) / p keys.
 * The splitting of stage 1 ranks r-1 splitters against p segments and the
 * rounds of stage 2 rank p/r - 1 splitters against p/r segments per group,
 * in place of p-1 splitters against p segments.
 */
typedef struct hss_staged_s* hss_staged_t;

/*
 * hss_staged_plan -- validate and prepare.  groups = r must divide p;
 * n, p, eps1, kt and tuning as for hss_plan (tuning: trace_level and
 * lsd_only must be zero, HSS_ERR_UNSUPPORTED otherwise; a probe budget
 * applies to both stages; the autotuner, when asked for, tunes stage 1);
 * 0 < eps2 < 1.  The plan holds
 * the workspace of stage 1, a staging buffer of N keys (and payload words),
 * and a cache of the device blocks of stage 2, whose layout depends on the
 * group sizes of each call.
 */
hss_status hss_staged_plan(hss_staged_t* out, uint64_t n, uint32_t p, uint32_t groups, double eps1,
                           double eps2, hss_key_type kt, int with_payload, const hss_tuning* tuning);

/* Release the plan and its device memory (synchronises the device). NULL is ok. */
void hss_staged_destroy(hss_staged_t plan);

/* Bytes of device memory held by the plan, its cached blocks included. */
size_t hss_staged_workspace_bytes(hss_staged_t plan);

/*
 * hss_staged_partition -- the two-stage partition.  Buffers as for
 * hss_partition (N keys in and out, payload words or NULL, p+1 offsets);
 * d_groups: NULL, or r+1 words that receive the group boundaries of stage
 * 1.  The host reads the r+1 group boundaries between the stages (one
 * synchronisation) to lay out stage 2.  A group with fewer than p/r keys
 * (possible only when N is close to p) gives HSS_ERR_UNSUPPORTED.  Returns
 * after the work on `stream` has completed.
 */
hss_status hss_staged_partition(hss_staged_t plan, uint64_t seed, const void* d_keys_in,
                                const uint64_t* d_vals_in, void* d_keys_out, uint64_t* d_vals_out,
                                uint64_t* d_offsets, uint64_t* d_groups, void* stream);

/*
 * hss_staged_sort -- the two-stage partition (section 5.3) followed by a
 * stable sort of every final bucket (the local sort after the last exchange):
 * d_keys_out (and d_vals_out) receive the keys in ascending order, equal keys
 * (with their payload) in input order; d_offsets and d_groups as for
 * hss_staged_partition.  The plan keeps a second buffer of N keys (and
 * payload words) from the first sort on, and reads the p+1 final offsets
 * back once to bound the bucket sort.  Errors as hss_staged_partition.
 */
hss_status hss_staged_sort(hss_staged_t plan, uint64_t seed, const void* d_keys_in, const uint64_t* d_vals_in,
                           void* d_keys_out, uint64_t* d_vals_out, uint64_t* d_offsets, uint64_t* d_groups,
                           void* stream);

/* Host wall time of the last call, in seconds: stage 1 (with the read of the
 * group boundaries), the layout of stage 2, stage 2. */
hss_status hss_staged_times(hss_staged_t plan, double* stage1_s, double* setup_s, double* stage2_s);

/*
 * hss_stream_copy -- measurement aid: copies `bytes` (a multiple of 16) from
 * src to dst (device pointers, 16-byte aligned, not overlapping) with 16-byte
 * loads and stores per lane, `workgroups` workgroups of 256 threads striding
 * over the buffer (1..65536), optionally with non-temporal loads and stores.
 * Its rate is the achievable HBM bandwidth the streaming kernels are compared
 * with.  Enqueued on `stream`; returns at once.  Errors: HSS_ERR_INVALID_ARG
 * for bad sizes or pointers (nothing enqueued), HSS_ERR_DEVICE if the launch
 * fails.
 */
hss_status hss_stream_copy(void* dst, const void* src, size_t bytes, uint32_t workgroups,
                           int nontemporal, void* stream);

const char* hss_status_string(hss_status status);

/* Message of the last failure on the calling thread ("" if none). */
const char* hss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HSS_H */
