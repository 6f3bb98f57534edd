/*
 * msf.h -- C ABI of the MI355X (gfx950) minimum spanning forest library.
 *
 * Computes the minimum spanning forest (MSF) of an undirected weighted
 * multigraph: a minimum spanning tree of every connected component (paper
 * Sec. II-B).  Ties between equal weights are broken by edge id, i.e. edge e
 * precedes edge f iff (w_e, e) < (w_f, f); under this strict order the MSF is
 * unique (Sec. II-C), so results are exact and reproducible bit for bit.
 *
 * Two algorithms are provided:
 *   MSF_ALGO_BORUVKA  Borůvka rounds (Sec. II-C, Alg. 1's round body):
 *                     lightest incident edge per vertex, 2-cycle tie break,
 *                     pointer jumping to stars, contraction to dense labels,
 *                     relabelling with self-loop removal.
 *   MSF_ALGO_FILTER   Filter-Borůvka (Sec. V, Alg. 2): sampled pivot, split
 *                     into light and heavy edges, recursion on the light ones,
 *                     removal of heavy edges inside a light component using the
 *                     representative array P, recursion on the survivors.
 *
 * Conventions shared by every entry point
 *   - Vertex ids are 0-based in [0, n) (the paper numbers them 1..|V|).
 *   - Edge e is (u[e], v[e], w[e]), undirected, listed once; its id is e.
 *     Self-loops and parallel edges are legal input.  A graph that lists both
 *     directions of an edge simply has two parallel edges; the lower id wins.
 *   - Limits: 0 <= n <= 2^31-1, 0 <= m <= 2^32-1, n == 0 requires m == 0.
 *   - Array arguments are DEVICE pointers (hipMalloc / torch tensors on ROCm)
 *     unless marked HOST.  Inputs are never modified.  The caller owns every
 *     buffer; the library writes only the outputs and the workspace.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).
 *   - Functions return an msf_status; nothing aborts or throws across the ABI.
 *     Argument errors are reported before any GPU work is launched.
 */
#ifndef MSF_H
#define MSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSF_OK = 0,
    MSF_EINVAL = -1,      /* bad argument (null pointer, n/m out of limits, bad options) */
    MSF_ERANGE = -2,      /* some u[e] or v[e] outside [0, n); outputs unspecified */
    MSF_ENOMEM = -3,      /* device allocation of an internal workspace failed */
    MSF_EDEVICE = -4,     /* a HIP call failed; msf_last_error() has the text */
    MSF_EWORKSPACE = -5,  /* caller workspace smaller than msf_workspace_bytes() */
    MSF_EINTERNAL = -6    /* an internal consistency check failed (a library bug) */
} msf_status;

typedef enum { MSF_ALGO_BORUVKA = 0, MSF_ALGO_FILTER = 1 } msf_algo;

typedef enum {
    MSF_PIVOT_MEDIAN = 0,    /* lower median of the sample (the paper's choice, Sec. V) */
    MSF_PIVOT_QUANTILE = 1,  /* sample quantile `quantile` in [0, 1] */
    MSF_PIVOT_MLP = 2        /* quantile predicted by the loaded pivot network;
                                falls back to the median when none is loaded */
} msf_pivot;

/* How round 0 runs when the graph is the caller's edge list (Sec. II-C's
 * lightest-edge search and relabelling):
 *   MSF_ROUND0_AUTO     by vertex buckets where the graph qualifies (2^21 <= n <= 2^24,
 *                       2^22 <= m < 2^31) and, in a sample of 4096 edges, at most half
 *                       join ids less than 2^14 apart; else on the edge list;
 *   MSF_ROUND0_EDGES    on the edge list, with random accesses into n-sized tables
 *                       (the workspace then holds no bucket buffers);
 *   MSF_ROUND0_BUCKETS  by vertex buckets wherever the graph qualifies.
 * By buckets, the edges are split once into per-endpoint arcs grouped by 2^14-vertex
 * buckets; the minimum and the relabelling then work on one bucket's vertices in LDS.
 * It costs msf_workspace_bytes about 24 extra bytes per edge and 8 per vertex. */
typedef enum { MSF_ROUND0_AUTO = 0, MSF_ROUND0_EDGES = 1, MSF_ROUND0_BUCKETS = 2 } msf_round0;

/* Parallel-edge removal (Sec. II-C makes it optional; Sec. VI-B filters with a
 * hash table before sorting).  Only the lightest edge of a vertex pair can be
 * in the MSF, so removing the others never changes the result:
 *   MSF_DEDUP_AUTO   the per-tile prefilter on graphs whose ids show locality
 *                    (a sample of 4096 edges, at least half joining ids less
 *                    than 2^14 apart), where contracted components share many
 *                    edges: round 0 then compacts the relabelled edges and every
 *                    later round compacts with the prefilter; otherwise NEVER;
 *   MSF_DEDUP_NEVER  parallel edges stay until the last pass before the
 *                    single-workgroup tail (which keeps one edge per pair);
 *   MSF_DEDUP_EXACT  every compaction keeps exactly the lightest edge of each
 *                    vertex pair, through a global hash table (needs
 *                    msf_workspace_bytes with this option: 32 more bytes per edge);
 *   MSF_DEDUP_LOCAL  the per-tile prefilter at every compaction (an LDS hash
 *                    table per tile of 2048 edges keeps the lightest edge of
 *                    each pair in the tile), whatever the ids look like. */
typedef enum { MSF_DEDUP_AUTO = 0, MSF_DEDUP_NEVER = 1, MSF_DEDUP_EXACT = 2,
               MSF_DEDUP_LOCAL = 3 } msf_dedup;

/* Options; a NULL pointer means {MSF_ALGO_BORUVKA, MSF_PIVOT_MEDIAN, 0.5, seed 1,
 * defaults}.  Every field only changes running time, never the result. */
typedef struct msf_options {
    int32_t algo;            /* msf_algo */
    int32_t pivot;           /* msf_pivot (filter only) */
    float quantile;          /* MSF_PIVOT_QUANTILE: sample quantile in [0, 1] */
    int32_t sample_size;     /* filter pivot sample size in [1, 8192]; 0 = 4096 */
    uint64_t seed;           /* seed of the pivot sampler's counter-based generator */
    int32_t sparse_degree;   /* filter isSparse: stop splitting when 2m'/n' <= this; 0 = 4 */
    int32_t min_split_edges; /* filter isSparse: stop splitting below this many edges; 0 = 2^20 */
    int32_t round0;          /* msf_round0: how round 0 on the caller's arrays is organised */
    int32_t dedup_policy;    /* msf_dedup: parallel-edge removal in the rounds */
    int32_t split_retries;   /* filter: balanced-split retry (proof of Thm. 1): a split
                                whose light fraction is more than 1/6 from the target
                                quantile (for the median: a side outside [|E|/3,
                                2|E|/3]) is drawn again, at most this many times per
                                split (the last draw is kept); 0 = off */
    int32_t defer_edges;     /* filter: a recursion below the top whose filtered heavy
                                set has fewer edges than this hands it back to its
                                caller, which filters it again with its own heavy
                                edges (Sec. VI-C, further remarks); 0 = off */
    int32_t tail_threshold;  /* the single-workgroup tail takes over the remaining rounds
                                (Sec. II-C's rounds, on the lightest edge of every vertex
                                pair) once at most this many component labels are left,
                                1..1024 (1 = never); 0 = automatic: at most 1024 labels
                                and at most 65536 possible pairs (live edges or label
                                pairs, whichever is fewer) */
    int32_t reserved[3];     /* must be zero */
} msf_options;

#define MSF_MAX_TRACE 64

/* Per-call statistics (HOST struct, optional). */
typedef struct msf_stats {
    uint64_t total_weight;      /* same as *total_weight_out */
    uint64_t msf_edges;         /* number of MSF edges = n - #components */
    uint32_t rounds;            /* Borůvka rounds executed (all base cases summed) */
    uint32_t levels;            /* filter recursion calls that split (0 for Borůvka) */
    uint32_t base_cases;        /* Borůvka base-case calls (1 for plain Borůvka) */
    float pivot_q_used;         /* quantile used at the first split (filter), else 0 */
    /* First MSF_MAX_TRACE rounds, in execution order: */
    uint64_t round_live[MSF_MAX_TRACE];   /* vertices with an incident live edge */
    uint64_t round_edges[MSF_MAX_TRACE];  /* edges scanned by the round */
    uint64_t round_found[MSF_MAX_TRACE];  /* MSF edges found by the round */
    uint64_t filtered_in;       /* heavy edges entering filtering (filter only) */
    uint64_t filtered_out;      /* heavy edges surviving filtering (filter only) */
    /* Filter-Borůvka splits in depth-first order (first MSF_MAX_TRACE): */
    uint64_t split_edges[MSF_MAX_TRACE];  /* edges of the graph being split */
    uint64_t split_pivot[MSF_MAX_TRACE];  /* pivot key w << 32 | edge id */
    uint64_t split_light[MSF_MAX_TRACE];  /* edges with key <= pivot */
    uint64_t split_kept[MSF_MAX_TRACE];   /* heavy edges surviving the filter */
    float split_q[MSF_MAX_TRACE];         /* sample quantile used by the split */
    float top_features[16];     /* pivot-network features of the first split's sample */
    float split_features[MSF_MAX_TRACE][16];  /* the same for every traced split */
    uint64_t round_vertices[MSF_MAX_TRACE];   /* vertex labels of each traced round (n_r) */
    uint32_t split_attempts[MSF_MAX_TRACE];   /* pivot draws of each split (retry) */
    uint64_t split_deferred_in[MSF_MAX_TRACE]; /* edges handed back by the light recursion */
    uint32_t pivot_retries;     /* redraws over the call */
    uint32_t deferrals;         /* filtered sets handed back to a caller */
} msf_stats;

/* Bytes of device workspace msf_compute needs for (m, n, opt); opt may be NULL. */
size_t msf_workspace_bytes(int64_t m, int64_t n, const msf_options* opt);

/*
 * msf_compute -- MSF of one graph.
 *   u, v, w       device arrays of length m (int32, int32, uint32), read only
 *   mask_out      device uint8[m]; on MSF_OK mask_out[e] = 1 iff edge e is in
 *                 the MSF, else 0
 *   total_weight_out  HOST; sum of w over MSF edges (cannot overflow 64 bits)
 *   workspace     device buffer of >= msf_workspace_bytes(m, n, opt) bytes,
 *                 256-byte aligned (hipMalloc and torch allocations are; else
 *                 MSF_EINVAL), or NULL: the library then allocates it on
 *                 `stream` and frees it before returning (MSF_ENOMEM if that
 *                 fails)
 *   stats         optional HOST struct, filled on MSF_OK
 * Blocking: returns once the mask and total are final.  Out-of-range ids are
 * detected on the device (such edges take no part in any minimum) and
 * reported as MSF_ERANGE after the first round.
 */
int msf_compute(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
                uint8_t* mask_out, uint64_t* total_weight_out, void* workspace,
                size_t workspace_bytes, void* stream, const msf_options* opt,
                msf_stats* stats);

/*
 * msf_compute_noalloc -- msf_compute for callers that cannot allocate device
 * memory: code that must not call hipMalloc (tight serving loops, harnesses
 * that forbid allocation, callers preparing work for stream capture).  The
 * workspace is a library-owned static device array of
 * MSF_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, obtained once
 * per GPU on the first call there and held until the process ends; the host
 * counter block is ordinary host memory; the kernel-timing profiler is not
 * used.  Nothing is allocated by the call.
 *   u, v, w, m, n, mask_out, total_weight_out, opt, stats: as msf_compute
 *   stream        a hipStream_t of the CURRENT device (the scratch copy used
 *                 is the current device's)
 * Limit: msf_workspace_bytes(m, n, opt) must not exceed
 * MSF_NOALLOC_SCRATCH_BYTES (e.g. plain Borůvka on up to about 2.6 million
 * edges plus vertices), else MSF_EWORKSPACE with the sizes in
 * msf_last_error().  Every call on one GPU uses that GPU's one array, whose
 * contents persist from call to call (each call clears what it needs), so two
 * overlapping calls on one GPU would race: the library serialises its own
 * calls per GPU with a host lock, and the caller must not run other work on
 * the array.  Blocking, like msf_compute.
 */
#define MSF_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int msf_compute_noalloc(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                        int64_t n, uint8_t* mask_out, uint64_t* total_weight_out, void* stream,
                        const msf_options* opt, msf_stats* stats);

/*
 * Batched MSF: G independent graphs solved by one persistent kernel (graph g
 * is a whole problem in the sense of msf_compute; all paper Sec. II-C rounds
 * run inside the kernel).  A graph with at least coop_edges edges is solved
 * by all workgroups running on one XCD together (one such graph per XCD at a
 * time); any other graph by one workgroup, with its state in LDS when it has
 * at most lds_vertices vertices.  Stream-ordered and asynchronous: nothing is
 * synchronised and nothing is allocated, so the call can be captured in a
 * hipGraph (see msf_batched_graph_create).  Calls sharing a workspace must
 * not overlap.
 *   u, v, w        device arrays of all graphs' edges, concatenated
 *   edge_off       device int64[G + 1]: graph g owns edges [edge_off[g], edge_off[g+1])
 *   vert_off       device int64[G + 1]: graph g has vert_off[g+1] - vert_off[g]
 *                  vertices; its u, v are LOCAL ids in [0, n_g)
 *   max_n          HOST: upper bound of n_g over the batch (sizes the scratch)
 *   order          device int32[G] processing order (e.g. largest first), or NULL
 *   mask_out       device uint8[edge_off[G]]: 1 iff the edge is in its graph's MSF
 *   totals_out     device uint64[G]: MSF weight per graph; UINT64_MAX marks a graph
 *                  with an id outside [0, n_g), n_g > max_n or more than 2^32-1 edges
 *   ticks_out      device uint64[2G + 1] or NULL: wall-clock ticks (rate:
 *                  msf_wall_clock_khz): [g] = graph g finished, [G] = the batch
 *                  started, [G + 1 + g] = graph g was taken up by a workgroup
 *                  (its service time is [g] - [G + 1 + g])
 *   workspace      device, >= msf_batched_workspace_bytes(G, max_n, opt) bytes,
 *                  256-byte aligned (else MSF_EINVAL)
 * Errors: MSF_EINVAL (bad host arguments), MSF_EWORKSPACE, MSF_EDEVICE.
 */
typedef struct msf_batch_options {
    int32_t block;           /* threads per workgroup: 256, 512 or 1024; 0 = 512 */
    int32_t lds_vertices;    /* graphs with at most this many vertices keep their
                                state in LDS (20 B per vertex); 0 = 8000, -1 = never */
    int32_t workgroups;      /* persistent workgroups; 0 = as many as can be resident */
    int32_t coop_edges;      /* graphs with at least this many edges are solved
                                cooperatively per XCD; 0 = 2^20, -1 = never */
    int32_t wave_edges;      /* a tier solving graphs with at most this many edges by
                                one wave each; SWITCHED OFF: only 0 and -1 (never) are
                                accepted, any positive value gives MSF_EINVAL */
    int32_t hot_min;         /* block tier of the lightest-edge search: a label on at
                                least this many of 64 sampled edge ends of a chunk
                                keeps its minimum in LDS for the chunk; 0 = 8,
                                -1 = off (1..64) */
    int32_t wave_min;        /* wave tier: lanes of a wave sharing a label are
                                min-reduced before updating when at least this many
                                share it; 0 = 2, -1 = off (2..64) */
    int32_t reserved[1];     /* must be zero */
} msf_batch_options;

size_t msf_batched_workspace_bytes(int64_t G, int64_t max_n, const msf_batch_options* opt);
int msf_compute_batched(const int32_t* u, const int32_t* v, const uint32_t* w,
                        const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                        int64_t max_n, const int32_t* order, uint8_t* mask_out,
                        uint64_t* totals_out, uint64_t* ticks_out, void* workspace,
                        size_t workspace_bytes, void* stream, const msf_batch_options* opt);

/* The same launch captured once into an instantiated hipGraph (fixed
 * arguments); launching it replays the whole batch. */
typedef struct msf_batch_graph msf_batch_graph;
int msf_batched_graph_create(const int32_t* u, const int32_t* v, const uint32_t* w,
                             const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                             int64_t max_n, const int32_t* order, uint8_t* mask_out,
                             uint64_t* totals_out, uint64_t* ticks_out, void* workspace,
                             size_t workspace_bytes, const msf_batch_options* opt,
                             msf_batch_graph** graph_out);
int msf_batched_graph_launch(msf_batch_graph* graph, void* stream);
int msf_batched_graph_destroy(msf_batch_graph* graph);

/*
 * Autotuner for the batched solver: a coordinate search from the defaults,
 * one option at a time in this order, keeping the fastest value of each:
 * block {512, 1024}, lds_vertices {1024, 2048, 4096, 8000}, coop_edges {2^18,
 * 2^19, 2^20, never}, hot_min {4, 8, 16, off}, wave_min {2, 4, off}.  Each candidate runs the batch once on `stream`, timed
 * with HIP events (after one warm-up run); the fastest options go to
 * *best_out (HOST) and its time to *best_ms_out (HOST, nullable).  Blocking.
 * Same array arguments as msf_compute_batched; the workspace must fit every
 * candidate (msf_batched_workspace_bytes with a NULL options pointer suffices).
 */
int msf_batched_autotune(const int32_t* u, const int32_t* v, const uint32_t* w,
                         const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                         int64_t max_n, const int32_t* order, uint8_t* mask_out,
                         uint64_t* totals_out, void* workspace, size_t workspace_bytes,
                         void* stream, msf_batch_options* best_out, float* best_ms_out);

/*
 * Pivot network for Filter-Borůvka (MSF_PIVOT_MLP).  Not in the paper, which
 * uses the sample median: a 16 -> 64 -> 64 -> 1 perceptron (ReLU hidden
 * layers, logistic output) maps 16 statistics of the pivot sample (listed in
 * filter.hip) to the sample quantile used as pivot, clamped to
 * [2^-10, 1 - 2^-10].  Any pivot yields the same MSF; the network only
 * changes running time.  Inference uses bfloat16 weights and activations with
 * FP32 accumulation.  Parameters are FP32 in the order W1[64][16], b1[64],
 * W2[64][64], b2[64], w3[64], b3 (msf_mlp_param_count() floats).
 */
/* Loads a model (HOST blob: uint32 magic 0x5046534d, version 1, 16, 64, then
 * the FP32 parameters).  MSF_EINVAL on a malformed blob or non-finite values.
 * Process-wide; later MSF_PIVOT_MLP solves use it. */
int msf_pivot_model_load(const void* blob, size_t bytes);
int msf_pivot_model_clear(void);          /* back to the median fallback */
int msf_pivot_model_loaded(void);         /* 1 if a model is loaded */
int msf_mlp_param_count(void);
/* Training kernels (all pointers DEVICE, stream-ordered):
 *   forward: z_out[b] = network output before the logistic, x is [B][16]
 *   grad:    grad_out[P] = d/dparams of mean_b (z_b - target_b)^2 / 2 and
 *            *loss_out = that loss (both overwritten); FP32 gradients
 *   adam:    one Adam step (Kingma & Ba) on FP32 params with moments m, v;
 *            step counts from 1
 * bf16 != 0 rounds weights, inputs and activations to bfloat16 in the forward
 * pass (accumulation stays FP32). */
int msf_mlp_forward(const float* params, const float* x, int64_t B, float* z_out, int bf16,
                    void* stream);
int msf_mlp_grad(const float* params, const float* x, const float* target, int64_t B, int bf16,
                 float* grad_out, float* loss_out, void* stream);
int msf_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, float beta1,
                 float beta2, float eps, int step, void* stream);

/* Rate of the device wall clock used by ticks_out, in kHz. */
int msf_wall_clock_khz(void);

/* Static description of a status code. */
const char* msf_status_string(int status);

/* Text of the last MSF_EDEVICE / MSF_EINTERNAL error on the calling thread. */
const char* msf_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int msf_version(void);

/*
 * Kernel timing for benchmarks.  While enabled, every kernel launch of
 * msf_compute is bracketed by HIP events recorded on the call's stream; the
 * elapsed times are accumulated per kernel together with the algorithmic
 * bytes of each launch (bytes the step must read or write at minimum, e.g.
 * 12 B per input edge for the first lightest-edge pass).  Process-wide state,
 * guarded by a lock; costs one event pair per launch.
 */
typedef struct msf_kernel_profile {
    char name[32];           /* kernel family */
    uint64_t launches;       /* launches timed */
    double total_ms;         /* summed event-timed duration */
    double bytes;            /* summed algorithmic bytes */
} msf_kernel_profile;

int msf_profile_enable(int on);                            /* returns MSF_OK */
int msf_profile_reset(void);                               /* returns MSF_OK */
/* Copies up to `capacity` entries (HOST array); returns the number copied. */
int msf_profile_read(msf_kernel_profile* out, int capacity);

#ifdef __cplusplus
}
#endif
#endif /* MSF_H */
