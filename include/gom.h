/*
 * gom.h -- C ABI of libgom: parallel Gene-pool Optimal Mixing (GOM) with partial evaluations
 * on weighted Max-Cut, parallelised by colouring the linkage-model interaction graph, on
 * AMD Instinct MI355X (gfx950).
 *
 * Paper: A. Bouter, P.A.N. Bosman, "GPU-Accelerated Parallel Gene-pool Optimal Mixing in a
 * Gray-Box Optimization Setting", arXiv 2203.08680.
 *
 * Conventions shared by every entry point:
 *  - Every call returns an int status: GOM_OK (0) or a negative GOM_E_* code.  No C++
 *    exception crosses this boundary.  gom_last_error() gives a message for the last failure
 *    on the calling thread.
 *  - On failure, outputs are left untouched and handles are unchanged.
 *  - Host arrays passed in are borrowed for the duration of the call (copied when kept).
 *  - Handles are owned by the caller and released with the matching *_free call.
 *  - Calls on different handles may run on different host threads at the same time; calls
 *    on one handle (and on the states of one batch or server) must not overlap.
 *  - Device memory is owned by the caller: a state lives inside a caller-provided device
 *    arena of gom_state_bytes() bytes (for example a torch uint8 tensor).  The library never
 *    allocates device memory.  `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream); all device work is enqueued on it.
 *  - Vertices are 0-based.  Genes are bits: gene 1 puts the vertex on one side of the cut,
 *    gene 0 on the other (the paper's x in {-1, 1}).
 */
#ifndef GOM_H
#define GOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mc_graph mc_graph;
typedef struct gom_fos gom_fos;
typedef struct gom_state gom_state;

enum {
    GOM_OK = 0,
    GOM_E_ARG = -1,    /* null pointer, bad enum, inconsistent sizes */
    GOM_E_GRAPH = -2,  /* invalid graph: vertex out of range, self-loop, repeated edge */
    GOM_E_RANGE = -3,  /* size outside what this build supports */
    GOM_E_NOMEM = -4,  /* host allocation failed, or the arena is too small */
    GOM_E_DEVICE = -5, /* a HIP call failed (message names it) */
    GOM_E_STATE = -6   /* call not valid in the handle's current state (e.g. not coloured) */
};

enum { GOM_FOS_UNIVARIATE = 0, GOM_FOS_NEIGHBOURHOOD = 1 };
enum { GOM_NEUTRAL_PAPER = 0, GOM_NEUTRAL_ALWAYS = 1 };
enum { GOM_ORDER_RANDOM = 0, GOM_ORDER_FIXED = 1 };

/* Largest population one state holds: one 64-bit population word per vertex. */
#define GOM_MAX_POP 64

/* Message for the last failed call on this thread ("" if none). */
const char *gom_last_error(void);

/* ABI version (incremented on incompatible changes). */
int gom_version(void);

/*
 * Weighted Max-Cut instance (Section 6.2: a graph G = (V, E) with a weight w(i, j) per edge).
 * Because w is a function of the vertex pair, the graph must be simple.
 *   n_vertices  number of vertices (>= 1)
 *   n_edges     number of edges m (>= 1, 2m < 2^31)
 *   u, v        host int32[m] endpoints, each in [0, n_vertices)
 *   w           host int32[m] weights (any sign, |w| <= 2^31 - 1); NULL = all weights 1
 *   out         receives the new handle
 * Errors: GOM_E_ARG (null), GOM_E_RANGE (n < 1, m < 1, 2m >= 2^31, a weight of -2^31),
 * GOM_E_GRAPH (endpoint out of range, u == v, the same unordered pair twice).
 * The graph is stored as CSR with each row sorted by neighbour id; total weight in int64.
 */
int mc_graph_load(int32_t n_vertices, int64_t n_edges, const int32_t *u, const int32_t *v,
                  const int32_t *w, mc_graph **out);

/* Sizes of a graph: vertices, edges, sum of weights, maximum degree.  Any output may be NULL. */
int mc_graph_info(const mc_graph *g, int32_t *n, int64_t *m, int64_t *total_weight,
                  int32_t *max_degree);

/* CSR copy: row_ptr int32[n+1], col int32[2m], w int32[2m] (rows ascending by col). */
int mc_graph_csr(const mc_graph *g, int32_t *row_ptr, int32_t *col, int32_t *w);

void mc_graph_free(mc_graph *g);

/*
 * Family of subsets (FOS, the linkage model of Section 4.1): a list of variable sets that
 * together cover every variable.
 *   kind GOM_FOS_UNIVARIATE     set v = {v}, v = 0..n-1
 *   kind GOM_FOS_NEIGHBOURHOOD  set v = {v} + N(v) (the vertex and its neighbours), ascending
 * Errors: GOM_E_ARG (null, bad kind).
 */
int gom_fos_build(const mc_graph *g, int kind, gom_fos **out);

/*
 * FOS from explicit sets: set j holds vars[ptr[j] .. ptr[j+1]-1] (host int32 arrays,
 * ptr[0] = 0, ptr non-decreasing).  Errors: GOM_E_ARG (null, n_sets < 1, empty set, variable
 * out of range, a variable twice in one set, a variable in no set: the FOS must be complete).
 */
int gom_fos_from_sets(const mc_graph *g, int32_t n_sets, const int32_t *ptr,
                      const int32_t *vars, gom_fos **out);

/*
 * Fixed linkage tree (Section 4.1, the Linkage Tree built with UPGMA; with a bound, the
 * Bounded Fixed Linkage Tree; Section 6.1 uses the graph's weights as the similarity).
 * Similarity of two variables = |w| of the edge between them, 0 without an edge; similarity of
 * two clusters = the average over all member pairs.  Starting from the n single variables,
 * UPGMA repeatedly merges a pair of clusters with the largest average similarity, ties broken
 * by the smaller combined size, then by the lower cluster ids (variables are clusters
 * 0..n-1, merged clusters get n, n+1, ... in creation order).  bound > 0: only pairs whose
 * union has at most `bound` variables may merge, and the tree stops when none is left;
 * bound = 0: no limit.  The set of all n variables is never added.
 * Sets: set v = {v} for v < n, then the merged clusters in creation order, members
 * ascending.  Every set above the variables is the union of exactly two earlier sets.
 * Errors: GOM_E_ARG (null, bound = 1 or negative).
 */
int gom_fos_build_lt(const mc_graph *g, int32_t bound, gom_fos **out);

/* FOS sizes: number of sets, total members, largest set.  Outputs may be NULL. */
int gom_fos_info(const gom_fos *f, int32_t *n_sets, int64_t *n_members, int32_t *max_set);

/* Copy the sets out: ptr int32[n_sets+1], vars int32[n_members] (each set ascending). */
int gom_fos_get(const gom_fos *f, int32_t *ptr, int32_t *vars);

void gom_fos_free(gom_fos *f);

/*
 * Group the FOS into mutually independent sets (Section 5.2): the Linkage Model Interaction
 * Graph joins sets j and k when they share a variable or a graph edge joins a variable of one
 * to a variable of the other; it is coloured greedily with Welsh-Powell (sets in order of
 * decreasing LMIG degree, ties by increasing set index, each taking the smallest colour not
 * held by a conflicting set coloured before it).  The LMIG is never stored.
 * Colour classes are numbered by first appearance in that order.  The colouring is stored in
 * the FOS handle; *n_colours receives the number of classes k.
 */
int gom_colour(const mc_graph *g, gom_fos *f, int32_t *n_colours);

/* Read the colouring: colour_of_set int32[n_sets], class_ptr int32[k+1], class_elems
 * int32[n_sets] (class c = class_elems[class_ptr[c] .. class_ptr[c+1]-1], ascending).
 * Any output may be NULL.  GOM_E_STATE if gom_colour was not called. */
int gom_colour_get(const gom_fos *f, int32_t *colour_of_set, int32_t *class_ptr,
                   int32_t *class_elems);

/* Device arena bytes needed for a state of population `pop` on (g, f).  f must be coloured.
 * GOM_E_RANGE unless 2 <= pop <= GOM_MAX_POP. */
int gom_state_bytes(const mc_graph *g, const gom_fos *f, int32_t pop, size_t *bytes);

/*
 * Create a run of parallel GOMEA (Algorithm 3) on device memory:
 *   pop           population size N, 2..GOM_MAX_POP
 *   seed          64-bit seed of every random draw (initial population, class order, donors)
 *   neutral_rule  GOM_NEUTRAL_PAPER: accept a step when the fitness rises, or stays equal
 *                 and the solution (at the start of the generation) differs from the
 *                 elitist (Section 5.3); GOM_NEUTRAL_ALWAYS: accept whenever it does not fall
 *   class_order   GOM_ORDER_RANDOM: classes in a random order per generation (Algorithm 3);
 *                 GOM_ORDER_FIXED: ascending class index
 *   dev_arena     device pointer to >= gom_state_bytes() bytes, 256-byte aligned, owned by
 *                 the caller and kept alive until gom_state_free
 * The instance data are copied into the arena; g and f may be freed afterwards.  The initial
 * population (uniform random genes), its fitness and the elitist are computed on the device.
 * Returns after the device work of the initialisation has completed.
 * Errors: GOM_E_ARG, GOM_E_RANGE (pop outside 2..GOM_MAX_POP, or n >= 2^27 vertices),
 * GOM_E_STATE (f not coloured), GOM_E_NOMEM (arena too small or misaligned), GOM_E_DEVICE.
 */
int gom_state_init(const mc_graph *g, const gom_fos *f, int32_t pop, uint64_t seed,
                   int neutral_rule, int class_order, void *dev_arena, size_t arena_bytes,
                   void *stream, gom_state **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gom_state_init without a caller arena.  The state's
 * device memory is the library's static arena, a file-scope device array of
 * GOM_STATIC_ARENA_BYTES that every device the library runs on holds until the process ends.
 * Nothing is allocated through HIP (the run-scalar read-back buffer is ordinary host memory).
 * One such state per device at a time: the arena is shared by every call on that device and
 * keeps the last state's contents, so a second gom_state_init_static on a device whose static
 * state has not been freed fails with GOM_E_STATE; gom_state_free releases it.  Calls that use
 * the static state from several host threads at once race, as for any state.
 * Errors: as gom_state_init; GOM_E_RANGE also when gom_state_bytes exceeds
 * GOM_STATIC_ARENA_BYTES; GOM_E_STATE when the device's static arena is in use.
 */
#define GOM_STATIC_ARENA_BYTES ((size_t)64 << 20)
int gom_state_init_static(const mc_graph *g, const gom_fos *f, int32_t pop, uint64_t seed,
                          int neutral_rule, int class_order, void *stream, gom_state **out);

/*
 * Start the run again from a new initial population drawn with `seed` (Algorithm 3,
 * InitializePopulation, then the fitness of every solution and the initial elitist), keeping
 * the instance data already in the arena.  Generation and counters restart at 0.
 * Asynchronous: enqueued on `stream`.
 */
int gom_state_reseed(gom_state *s, uint64_t seed, void *stream);

/* Enqueue one generation (Algorithm 3: clone, every colour class in the generation's order,
 * then P <- O and the elitist update).  Asynchronous.  If gom_debug_stop_after_class left a
 * generation open, this finishes it (the remaining classes, then the generation end). */
int gom_generation(gom_state *s, void *stream);

/*
 * Debugging view between two groups of Algorithm 3: start the next generation if none is open,
 * run the colour classes of its order up to and including order position class_position, and
 * leave it open.  While it is open, gom_state_read and gom_state_hash show the offspring O,
 * the running fitness (generation-start fitness plus the accepted deltas so far) and running
 * counters; the generation counter and the elitist are unchanged.  The open part runs under
 * the class-launch schedule (bit-sliced when that is the chosen one); finishing with
 * gom_generation gives exactly the uninterrupted generation.  Asynchronous.
 * GOM_E_RANGE: class_position outside [0, n_classes).  GOM_E_STATE: the open generation has
 * already run that position.  gom_run_to_target, gom_state_autotune and gom_batch_run return
 * GOM_E_STATE while a generation is open; gom_state_write and gom_state_reseed close it.
 */
int gom_debug_stop_after_class(gom_state *s, int32_t class_position, void *stream);

/*
 * Colouring-parallel local search, the hybrid that the paper's conclusion names as future work
 * (colour classes are sets of independent variables, so their single-bit flips can be made
 * together).  For a state whose FOS is univariate (its colour classes are then those of the
 * graph), between generations: for every solution, a pass visits the colour classes in
 * ascending class index and flips each variable of the class whose flip strictly raises the
 * solution's fitness; passes repeat until one flips nothing in any solution or max_passes
 * passes have run.  Then the population is the searched one and the elitist is replaced when
 * the best solution (lowest index on ties) is strictly better, as at a generation end.  The
 * generation counter and the attempted/evaluated/accepted counters do not change.
 * Synchronous (one read-back per pass).  *passes (may be NULL): the passes run, counting the
 * last one that flipped nothing.
 * Errors: GOM_E_ARG (null state, max_passes < 0), GOM_E_STATE (FOS not univariate, or a
 * generation left open by gom_debug_stop_after_class), GOM_E_DEVICE.
 */
int gom_local_search(gom_state *s, int32_t max_passes, void *stream, int32_t *passes);

/*
 * Iterated local search around the search above (the conclusion's "(iterated)" hybrid; the
 * paper gives no procedure, so this is one reading of it).  Rounds round0 .. round0+rounds-1,
 * each for every solution i at once:
 *   perturbation: for t = 0 .. flips-1, word (t mod 4) of Philox4x32-10(key = seed, counter =
 *     (generation, 0xFFFFFFFE, i, 16 r + t / 4)) scaled to q = (word * n_sets) >> 32 names
 *     the set at position q of the colour-class order (classes in index order, sets ascending
 *     within a class); its variable flips in a copy of solution i, one flip after another;
 *   search: the passes of gom_local_search on the copies (at most max_passes);
 *   acceptance: solution i becomes its copy unless the copy's fitness is below its own;
 * then the elitist is replaced when the best solution is strictly better.  The generation and
 * the attempted/evaluated/accepted counters do not change.  Rounds are numbered so that
 * rounds [a, b) then [b, c) equal rounds [a, c); the same rounds at the same generation draw
 * the same flips.  Synchronous.  *passes (may be NULL): search passes summed over the rounds.
 * Errors: GOM_E_ARG (null state, round0 < 0, rounds < 0, round0 + rounds > 2^27, flips
 * outside 0..64, max_passes < 0), GOM_E_STATE (FOS not univariate, or a generation left open),
 * GOM_E_DEVICE.
 */
int gom_iterated_local_search(gom_state *s, int32_t round0, int32_t rounds, int32_t flips,
                              int32_t max_passes, void *stream, int32_t *passes);

typedef struct {
    int32_t generations; /* generations run by this call */
    int32_t reached;     /* 1 if the elitist fitness is >= target */
    int64_t best;        /* elitist fitness */
    int64_t attempted;   /* cumulative (solution, set) pairs visited: N * n_sets per generation */
    int64_t evaluated;   /* cumulative pairs that found a differing donor and were evaluated */
    int64_t accepted;    /* cumulative accepted steps */
} gom_result;

/*
 * The generation loop of Algorithm 3 with a stopping rule: run generations until the elitist
 * fitness is >= target or the state has run max_generations generations in total (the target
 * is also tested before the first one).  Section 6.4 measures the time until the known
 * optimum is reached, and Section 6.5 runs under a limit; target and max_generations are
 * those two conditions (the paper uses wall-clock limits; a generation count is used here so
 * that runs are reproducible).
 * Synchronous: returns when the device work has finished.  Generations are enqueued ahead in
 * small chunks; a generation enqueued after the target was reached does nothing on the device.
 * out (may be NULL) receives the generations run and the cumulative counters.
 * A max_generations at or below the generations already run runs none.
 * Errors: GOM_E_ARG (null state), GOM_E_STATE (a generation left open by
 * gom_debug_stop_after_class), GOM_E_DEVICE.
 */
int gom_run_to_target(gom_state *s, int64_t target, int32_t max_generations, void *stream,
                      gom_result *out);

/*
 * Copy the state to the host (synchronous): the population P of Algorithm 3 (between
 * generations; the offspring O while gom_debug_stop_after_class holds a generation open), the
 * fitness of every solution (Section 6.2 objective), the elitist of Section 4 (the best
 * solution found so far) with its fitness, the generation counter and the step counters:
 *   genes         uint8[N * n] solution-major (genes[i*n + v]) or NULL
 *   fitness       int64[N] or NULL
 *   elite         uint8[n] or NULL; elite_fitness, generation: or NULL
 *   counters      int64[3] {attempted, evaluated, accepted} or NULL
 */
int gom_state_read(gom_state *s, void *stream, uint8_t *genes, int64_t *fitness, uint8_t *elite,
                   int64_t *elite_fitness, int32_t *generation, int64_t *counters);
/* Errors: GOM_E_ARG (null state), GOM_E_DEVICE (a copy failed; outputs may then be partly
 * written). */

/*
 * 64-bit summary of the whole state, for comparing runs generation by generation without
 * copying populations (synchronous).  Canonical byte string: the genes solution-major (N*n
 * bytes, 0/1), the N fitness values (8 little-endian bytes each), the elitist's n genes, the
 * elitist fitness (8), the generation (4), attempted, evaluated, accepted (8 each) -- the
 * values gom_state_read returns.  hash = sum modulo 2^64 over byte positions k of
 * M(256*k + b_k), M = the output mixer of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).
 * The gene and elitist terms are summed on the device.
 */
int gom_state_hash(gom_state *s, void *stream, uint64_t *hash);

/*
 * Overwrite the state (resume from a checkpoint): genes uint8[N*n] (0/1), elite uint8[n],
 * the elitist fitness, the generation counter and counters {attempted, evaluated, accepted}.
 * Fitness is recomputed on the device.  GOM_E_ARG for a gene outside {0, 1}.
 */
int gom_state_write(gom_state *s, void *stream, const uint8_t *genes, const uint8_t *elite,
                    int64_t elite_fitness, int32_t generation, const int64_t *counters);

/*
 * Kernel timing: with period k > 0, every k-th sweep launch (the colour-class sweeps, or the
 * resident generation sweep) records a pair of HIP events with its own dispatch
 * (hipExtLaunchKernelGGL), so the elapsed time is the kernel's execution from its start to
 * its end on the device; k = 0 turns timing off.  gom_timing_read
 * waits for the recorded events, returns the summed elapsed milliseconds and the number of
 * timed launches since the last read, and resets them.
 */
int gom_timing_enable(gom_state *s, int period);
int gom_timing_read(gom_state *s, double *class_ms_total, int64_t *class_launches);

/*
 * Launch schedule of a state's generations (results are identical under every schedule):
 *   GOM_SCHED_CLASS_LAUNCH  one kernel launch per colour class, each covering every
 *                           (solution, set) pair of the class; suits large instances
 *   GOM_SCHED_RESIDENT      one launch per generation, one workgroup per solution holding its
 *                           offspring in LDS and running all classes with barriers between
 *                           them; needs n bytes of LDS per workgroup and at most
 *                           GOM_RESIDENT_MAX_CLASSES classes
 *   GOM_SCHED_BITSLICED     one launch per colour class, lane = set, the solutions of the
 *                           set as the bits of machine words.  Univariate FOS: every class,
 *                           all solutions at once with 64-bit bitwise operations; needs
 *                           maximum degree <= 4 and per-vertex sums of |w| below 2^30.
 *                           General FOS (population <= 64): the classes whose sets have at
 *                           most 9 members, per-set sums of |w| over their dependent edges of
 *                           at most 16383 and at least gom_state_set_bitsliced_min_sets sets
 *                           (default 32768): per solution the donor draw and the changed
 *                           members, then the fitness changes of 32 solutions at once as a
 *                           bit-sliced sum; the other classes as under class launch
 *   GOM_SCHED_AUTO          resident when it fits the device and the instance has at most
 *                           1536 vertices (larger ones run faster spread over the device
 *                           by class), else bit-sliced when the instance qualifies
 *                           (univariate, or general with a class of at least the bit-sliced
 *                           threshold), else class launch
 * GOM_E_RANGE when the requested schedule does not fit this instance or device.
 */
enum { GOM_SCHED_AUTO = 0, GOM_SCHED_CLASS_LAUNCH = 1, GOM_SCHED_RESIDENT = 2,
       GOM_SCHED_BITSLICED = 3 };
#define GOM_RESIDENT_MAX_CLASSES 1536
int gom_state_set_schedule(gom_state *s, int schedule);
/* The schedule in use (GOM_SCHED_CLASS_LAUNCH, GOM_SCHED_RESIDENT or GOM_SCHED_BITSLICED). */
int gom_state_get_schedule(const gom_state *s, int *schedule);

/*
 * Forced improvement (Section 4 describes the serial procedure; Section 5.4 leaves a parallel
 * form open), off by default as in the paper's parallel GOMEA.  When on, after each
 * generation's classes every solution that had no accepted GOM step takes GOM steps with the
 * elitist (of the generation start) as donor, class by class in the generation's order, all
 * sets of a class together; it stops after the first class in which its fitness rose, and is
 * replaced by a copy of the elitist if it never did.  With one set per class this is the
 * serial procedure.  These steps count in `evaluated` and `accepted` (not in `attempted`).
 * The bit-sliced schedule has no forced improvement: turning it on moves a bit-sliced state
 * to the automatic choice among the others.  GOM_E_STATE while a generation is open.
 */
int gom_state_set_fi(gom_state *s, int enabled);
int gom_state_get_fi(const gom_state *s, int *enabled);

/* Block size of the class-launch sweeps: 64..512 threads, a multiple of 64 (default 256).
 * GOM_E_RANGE otherwise.  Results do not depend on it. */
/*
 * The fused form of the bit-sliced schedule: a whole generation's classes in one cooperative
 * launch, each block waiting only for the chunks of earlier classes whose sets conflict with
 * its own (same variable or an edge between them; Sec. 5.2's independence of the sets of a
 * colour class).  Available when the bit-sliced schedule is, there are at most 8 classes and
 * every dependency range spans at most 32 chunks (tori, not random graphs); off by default:
 * each block's device-scope release and acquire write back and invalidate its L2, which on
 * the 10^6- and 10^7-vertex tori cost more than the per-class launches save (220 against 37
 * and 520 against 232 us per generation).  Results are identical either way.  Its blocks wait for each other, so they must all
 * be on the device at once: the launch is cooperative, and states that generate on several
 * streams at the same time should turn it off (the serving loop does for its jobs).  A
 * dependency wait that never ends gives up after a bounded number of polls; the next read of
 * the state then fails with GOM_E_DEVICE.
 * gom_state_set_fused errors: GOM_E_ARG, GOM_E_RANGE (not available).
 */
int gom_state_set_fused(gom_state *s, int enabled);
/*
 * Grid cap (blocks) of the per-class sweeps (default 2048): a class larger than the cap's
 * threads is swept with each group striding over several positions.  For tuning and tests;
 * results do not depend on it.  Errors: GOM_E_ARG, GOM_E_RANGE (outside 1..65536).
 */
int gom_state_set_grid_limit(gom_state *s, int32_t blocks);
/*
 * Smallest class (sets) that the bit-sliced schedule sweeps with the general bit-sliced
 * sweep (general FOS; default 32768: one set per lane leaves a smaller class too few waves).
 * Results do not depend on it.  A state under the bit-sliced schedule that no class
 * qualifies for any more falls back to GOM_SCHED_AUTO's choice.
 * Errors: GOM_E_ARG, GOM_E_RANGE (negative).
 */
int gom_state_set_bitsliced_min_sets(gom_state *s, int32_t sets);
/*
 * Class sweeps of small general sets (at most 9 members and 72 dependent edges; population
 * above 32) stage each set in two rounds of loads by its wave (record, then member and
 * far-end words) instead of fetching the record's entries in batches (default off: on the
 * 100x100 torus's neighbourhoods it was 7 % slower per generation, on the 10^6-vertex torus's
 * within 1 %).  Results are identical either way.  Errors: GOM_E_ARG.
 */
int gom_state_set_staged(gom_state *s, int enabled);
int gom_state_get_fused(const gom_state *s, int *enabled, int *available);
int gom_state_set_block(gom_state *s, int threads);
int gom_state_get_block(const gom_state *s, int *threads);

/*
 * Autotuner: for every candidate this instance allows (class launch with blocks of 64, 128,
 * 256 and 512 threads, resident, bit-sliced), one untimed generation and then
 * `trial_generations` generations timed with HIP events on `stream`; two interleaved rounds;
 * keeps the candidate (schedule and block size) with the fastest round.  The trial
 * generations are ordinary generations of the run (every schedule gives the same results), so
 * the state advances by 2 x (candidates) x (trial_generations + 1) generations.  *chosen (may
 * be NULL) receives the schedule kept.
 */
int gom_state_autotune(gom_state *s, int32_t trial_generations, void *stream, int *chosen);

/* Sizes of a state: vertices, population, sets, classes, largest class. */
int gom_state_info(const gom_state *s, int32_t *n, int32_t *pop, int32_t *n_sets,
                   int32_t *n_classes, int32_t *max_class);

/* Releases host resources of the state; the caller frees the arena afterwards. */
void gom_state_free(gom_state *s);

/*
 * Batches: many independent instances (each its own graph, FOS, population and seed) run in
 * lockstep, one generation step for all of them per group of launches:
 *   - sweep launches (one per group of instances with the same block size and blocks per
 *     compute unit, see gom_batch_set_narrow) with one workgroup per (instance, solution)
 *     running every colour class of that instance (the resident schedule; each workgroup
 *     draws its instance's class order from the instance's seed and generation);
 *   - a finalize launch with one wave per instance;
 *   - a vertex-pass launch over all instances' vertices.
 * Every instance follows exactly the trajectory it has when run alone with the same seed:
 * batching changes when work runs, not what is computed.  Instances whose elitist has reached
 * their target stop changing.  An instance beyond the resident schedule (its offspring bytes
 * do not fit in LDS, or more than GOM_RESIDENT_MAX_CLASSES classes) runs its own per-class
 * sweeps and epilogue within each step, with the schedule its state chooses (bit-sliced or
 * class launch); those launches are enqueued after the captured graph of a chunk.
 */
typedef struct gom_batch gom_batch;

/* Device arena bytes for a batch of `count` instances (graphs[b], fos[b] coloured, pops[b]). */
int gom_batch_bytes(int32_t count, const mc_graph *const *graphs, const gom_fos *const *fos,
                    const int32_t *pops, size_t *bytes);

/*
 * Create a batch in the caller's device arena (256-byte aligned, >= gom_batch_bytes bytes):
 * instance b gets population pops[b], seed seeds[b] and target targets[b] (the elitist
 * fitness at which it stops).  Neutral rule and class order as for gom_state_init.  Host
 * arrays are borrowed; graphs and FOS may be freed afterwards.  Synchronous.
 * Errors: GOM_E_ARG, GOM_E_RANGE (population outside 2..64), GOM_E_STATE (FOS not
 * coloured), GOM_E_NOMEM, GOM_E_DEVICE.
 */
int gom_batch_init(int32_t count, const mc_graph *const *graphs, const gom_fos *const *fos,
                   const int32_t *pops, const uint64_t *seeds, const int64_t *targets,
                   int neutral_rule, int class_order, void *dev_arena, size_t arena_bytes,
                   void *stream, gom_batch **out);

/*
 * Run generation steps until every instance has reached its target or the batch has run
 * max_generations steps in total.  Synchronous.  results (count entries, or NULL) as for
 * gom_run_to_target; time_to_target_ms (count entries, or NULL): device time from the start
 * of this call to the finalize that first reached the instance's target, or -1.
 */
int gom_batch_run(gom_batch *b, int32_t max_generations, void *stream, gom_result *results,
                  double *time_to_target_ms);

/*
 * How gom_batch_run enqueues its generation steps: as one captured HIP graph per chunk of 4
 * steps (enabled != 0, the default) or as separate kernel launches (enabled == 0).  The graph
 * holds the chunk's 12 kernels (sweep, finalize and vertex pass of each step) and the gather
 * of the instances' run scalars; it is captured on a private stream the first time it is
 * needed and replayed on the caller's stream.  Chunks shorter than 4 steps (the end of a
 * generation budget) are always launched directly.  Results are identical either way.
 * Errors: GOM_E_ARG (null batch).
 */
int gom_batch_set_graph(gom_batch *b, int enabled);

/*
 * Restart every instance from a fresh initial population (Algorithm 3, InitializePopulation:
 * the set-up step a0) drawn with seeds[b] (count entries, borrowed): population, full
 * fitness, elitist, generation 0 and zero counters, as gom_state_init would leave them.  The
 * step budget of gom_batch_run counts from 0 again.  Synchronous.
 * Errors: GOM_E_ARG, GOM_E_STATE (an instance has an open generation), GOM_E_DEVICE.
 */
int gom_batch_reseed(gom_batch *b, const uint64_t *seeds, void *stream);

/*
 * Kernel timing of the batched sweep: while enabled, gom_batch_run launches every step
 * directly (no graph) and the sweep launch of each step records a pair of HIP events with its
 * own dispatch.  gom_batch_timing_read waits for the recorded pairs and returns the summed
 * sweep time (ms) and the number of timed launches since the previous read, then resets both.
 * Errors: GOM_E_ARG, GOM_E_DEVICE.
 */
int gom_batch_timing_enable(gom_batch *b, int enabled);
int gom_batch_timing_read(gom_batch *b, double *sweep_ms_total, int64_t *sweep_launches);

/*
 * Block sizes of the batched sweep.  An instance with at most narrow_max_n vertices sweeps
 * with 256-thread blocks, a larger one with 1024-thread blocks; it keeps a copy of the
 * population words in LDS when that does not lower the number of its blocks a compute unit
 * holds.  Instances with the same block size and blocks per compute unit share one sweep
 * launch per step (longest blocks first).  Results do not depend on the choice.  Default
 * 16384.  Synchronous (uploads the block map).
 * gom_batch_get_narrow returns the threshold and the number of sweep launches per step.
 * Errors: GOM_E_ARG, GOM_E_RANGE (an instance's LDS does not fit), GOM_E_DEVICE.
 */
int gom_batch_set_narrow(gom_batch *b, int64_t narrow_max_n, void *stream);
int gom_batch_get_narrow(const gom_batch *b, int64_t *narrow_max_n, int32_t *launches);

/*
 * Batched class launches: instances of a general FOS whose sets all have at most 14 members
 * (neighbourhoods of graphs up to degree 13) and at least min_n vertices are swept per colour
 * class instead of by resident blocks: each step draws every such instance's class order on
 * the device, then launches once per class position t, every launch covering class pi_i[t]
 * of all of them with one wave per set and one lane per solution (Algorithm 3's loop over
 * groups, for many instances at once), so a set's record is read once for all solutions.
 * min_n < 0: none.  Default 20000.  Results do not depend on the choice.  Synchronous.
 * gom_batch_get_class_launch returns the threshold, the instances it selects and the class
 * launches per step.  Errors: GOM_E_ARG, GOM_E_DEVICE.
 */
int gom_batch_set_class_launch(gom_batch *b, int64_t min_n, void *stream);
int gom_batch_get_class_launch(const gom_batch *b, int64_t *min_n, int32_t *instances,
                               int32_t *launches, int32_t *positions_per_wave);
/* Consecutive class positions a wave of the class launches sweeps (1..8; default 2): more
 * share a Philox call, fewer give small classes more waves.  Errors: GOM_E_ARG, GOM_E_RANGE. */
int gom_batch_set_class_positions(gom_batch *b, int32_t positions_per_wave);
/*
 * Bit-sliced form of the class launches (default on where available): four lanes share each
 * half (32 solutions) of a set, over the sets of every class-launched instance's class at a
 * position, with the donor draws per solution and the fitness changes of 32 solutions as one
 * bit-sliced sum (as the bit-sliced schedule's general sweep).  Available when every general
 * instance that takes the class launches has per-set sums of |w| over the dependent edges of
 * at most 16383 and |w| of at most 13 bits.  In this form, univariate instances that the
 * univariate bit-sliced sweep fits (degree <= 4) take the class launches too, at the same
 * size threshold, one lane a set with all solutions in one word.  Results are identical
 * either way.  Regroups the batch (synchronous on `stream`).  gom_batch_get_class_bitsliced:
 * in use, available (either may be NULL).  Errors: GOM_E_ARG, GOM_E_DEVICE.
 */
int gom_batch_set_class_bitsliced(gom_batch *b, int enabled, void *stream);
int gom_batch_get_class_bitsliced(const gom_batch *b, int *enabled, int *available);

/*
 * Autotuner of the batch's launch shapes: runs trial_steps generation steps under each
 * candidate class-launch threshold (none, 50000, 20000, 5000 vertices, all eligible), then
 * under each block-size threshold (all 1024-thread blocks, 2048, 8192, 16384, 32768 vertices,
 * all 256-thread blocks), then (when some instance takes the class launches) the bit-sliced
 * form where available against 1, 2, 4 and 8 positions per wave of the lane-per-solution
 * form, candidates that give the same assignment only once, timed with HIP events on `stream`
 * in two interleaved rounds, and keeps the fastest of each.  The trial
 * steps are ordinary generation steps of the run (they count against gom_batch_run's step
 * budget).  Synchronous.  narrow, class_min (or NULL): the thresholds kept.
 * Errors: GOM_E_ARG, GOM_E_STATE (an open generation), GOM_E_RANGE, GOM_E_DEVICE.
 */
int gom_batch_autotune(gom_batch *b, int32_t trial_steps, void *stream, int64_t *narrow,
                       int64_t *class_min);

/* Borrowed handle of instance `index` (for gom_state_read); valid until gom_batch_free. */
int gom_batch_state(gom_batch *b, int32_t index, gom_state **state);

/* Releases the batch and its instances' host resources; the caller frees the arena. */
void gom_batch_free(gom_batch *b);

/* ------------------------------------------------------------------------------------------
 * Interleaved Multi-start Scheme (Section 6.3).  Level i (1-based) is a population of
 * n_base * 2^(i-1) solutions with seed `seed + i - 1`.  A step runs one generation of level
 * 1 and, whenever level i has then completed a multiple of c_ims generations, one generation
 * of level i + 1 (created, in its own part of the arena, when it first runs), up to
 * max_levels levels.  The run ends after the step in which some level's elitist reaches
 * `target`, or when max_total_generations generations have run.  Synchronous (the elitists
 * are read after every step).
 * ------------------------------------------------------------------------------------------ */
#define GOM_IMS_MAX_LEVELS 8

typedef struct {
    int32_t levels;             /* levels created */
    int32_t steps;              /* steps run */
    int32_t total_generations;  /* generations over all levels */
    int32_t reached;            /* 1 if some level's elitist reached the target */
    int64_t best;               /* best elitist fitness over the levels */
    int32_t best_level;         /* its level (1-based; the lowest on ties) */
    int32_t generations[GOM_IMS_MAX_LEVELS];  /* per level */
    int64_t evaluated, accepted;  /* summed over the levels */
} gom_ims_result;

/* Arena bytes for max_levels levels.  GOM_E_RANGE if n_base * 2^(max_levels-1) exceeds
 * GOM_MAX_POP; GOM_E_ARG for max_levels outside 1..GOM_IMS_MAX_LEVELS or n_base < 2. */
int gom_ims_bytes(const mc_graph *g, const gom_fos *f, int32_t n_base, int32_t max_levels,
                  size_t *bytes);

/* Run the scheme on (g, f coloured).  forced_improvement: 0/1 for every level.  states:
 * NULL, or an array of max_levels handles that receives the levels' states (NULL where a
 * level was not created); the caller then owns them (gom_state_free), and their memory is
 * in dev_arena. */
int gom_ims_run(const mc_graph *g, const gom_fos *f, int32_t n_base, int32_t c_ims,
                int32_t max_levels, uint64_t seed, int neutral_rule, int forced_improvement,
                int64_t target, int32_t max_total_generations, void *dev_arena,
                size_t arena_bytes, void *stream, gom_ims_result *out, gom_state **states);

/* ------------------------------------------------------------------------------------------
 * Serving loop with continuous batching.  Jobs (a graph, a coloured FOS, a population size, a
 * seed, a target and a generation limit) are submitted at any time and wait in a queue.
 * gom_server_step admits queued jobs first come first served while their states fit in the
 * server's arena (the HBM budget), and moves every admitted job forward without waiting for
 * the others: each job runs on one of the server's streams (the least loaded at admission),
 * in chunks of 4 generations under the schedule gom_state_init chose for it, two chunks in
 * flight (the next one queued while one runs); as soon as a chunk has finished the job is
 * retired once its last chunk is done (target or generation limit reached; its memory is
 * freed) or given another chunk.  Jobs on different streams overlap on the device.
 * A job's random numbers depend on its seed alone, so its result equals that of
 * gom_run_to_target on a fresh state with the same arguments, whatever else runs beside it.
 * ------------------------------------------------------------------------------------------ */
typedef struct gom_server gom_server;

typedef struct {
    int64_t job;          /* id from gom_server_submit */
    int32_t generations;  /* generations run */
    int32_t reached;      /* 1 if the elitist fitness reached the target */
    int64_t best;         /* elitist fitness */
    int64_t attempted, evaluated, accepted;
    uint64_t hash;        /* gom_state_hash of the final state */
    double submit_ms, admit_ms, done_ms;  /* host clock, ms since gom_server_create; done_ms
                                             is when a step found the job finished */
    int32_t status;       /* GOM_OK, or the error that kept the job from starting (its state
                             could not be created); the other fields are then 0 */
} gom_job_result;

/*
 * dev_arena: caller-owned device memory (256-byte aligned) in which admitted jobs' states are
 * placed first-fit.  max_jobs: most jobs admitted at once.  streams: number of streams the
 * server creates for its jobs (1..16, default priority).  Errors: GOM_E_ARG, GOM_E_NOMEM
 * (misaligned or too small), GOM_E_DEVICE.
 */
int gom_server_create(void *dev_arena, size_t arena_bytes, int32_t max_jobs, int32_t streams,
                      gom_server **out);

/*
 * Size-aware placement: a job whose graph has at least large_min_n vertices is large.  Large
 * jobs run one at a time, on the server's first stream, first come first served among
 * themselves; a large job that has to wait does not hold back the small jobs queued behind it,
 * which run on the other streams.  So a large job shares the device only with small ones,
 * and small jobs never queue behind large ones.  large_min_n < 0 (the default) or a server
 * with one stream: every job is placed on the least loaded stream.  Errors: GOM_E_ARG.
 */
int gom_server_set_large(gom_server *s, int64_t large_min_n);

/* Queue a job.  g and f (coloured) are borrowed: keep them alive until the job's result has
 * been returned.  *job receives its id (0, 1, ...).  Errors: as gom_state_bytes, GOM_E_NOMEM
 * if the job could never fit the arena, GOM_E_ARG. */
int gom_server_submit(gom_server *s, const mc_graph *g, const gom_fos *f, int32_t pop,
                      uint64_t seed, int64_t target, int32_t max_generations,
                      int neutral_rule, int class_order, int64_t *job);

/* One pass: admit what fits, retire or continue every job whose chunk has finished.  Returns
 * without waiting for running chunks (call it in a loop).  Outputs may be NULL.  A job whose
 * state cannot be created at admission leaves the queue with a result whose status is the
 * error.  On a device error the pass stops and returns GOM_E_DEVICE; jobs it had already
 * retired keep their results and the others stay admitted. */
int gom_server_step(gom_server *s, int32_t *n_active, int32_t *n_queued);

/* Move up to `capacity` finished jobs' results into out (in retirement order); *n receives
 * the number moved. */
int gom_server_results(gom_server *s, gom_job_result *out, int32_t capacity, int32_t *n);

/* Admitted jobs, queued jobs, streams, free arena bytes.  Outputs may be NULL. */
int gom_server_info(const gom_server *s, int32_t *n_active, int32_t *n_queued,
                    int32_t *n_streams, size_t *free_bytes);

/* Waits for the server's streams and releases it (jobs still admitted are dropped). */
void gom_server_free(gom_server *s);

#ifdef __cplusplus
}
#endif
#endif /* GOM_H */
