// gom_internal.h -- structures shared by the host driver (gom_host.cpp) and the kernels
// (gom_kernels.hip) of libgom.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gom {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), keyed by a 64-bit seed split into
// (low, high) words.  Ten rounds; each multiplies counter words 0 and 2 by the two round
// multipliers, swaps in the high halves xor-ed with the other words and the round key, and
// advances the key by the two Weyl increments.  Used on the host (class order) and on the
// device (initial population, donor draws).
struct U32x4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ U32x4 philox(uint64_t seed, uint32_t c0, uint32_t c1,
                                                 uint32_t c2, uint32_t c3) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {x0, x1, x2, x3};
}

// Output mixer of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state hash is the sum
// modulo 2^64 of mix64(256 k + b_k) over the bytes b_k of a canonical byte string.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Counter word values that keep the Philox streams apart: generation indices are below
// 0xFFFFFFFF and class indices below 0xFFFFFFFE.
constexpr uint32_t kInitStream = 0xFFFFFFFFu;   // counter (kInitStream, i, v/128, 0)
constexpr uint32_t kOrderStream = 0xFFFFFFFFu;  // counter (g, kOrderStream, t, 0)
constexpr uint32_t kPerturbStream = 0xFFFFFFFEu;  // counter (g, kPerturbStream, i, 16r + t/4)
constexpr int32_t kMaxPerturbRounds = 1 << 27;     // 16 r + t/4 stays below 2^32

// Per-run scalars.  The finalize kernel updates them once per generation.
struct alignas(64) DevState {
    int64_t elite_fitness;   // fitness of the elitist
    int64_t evaluated;       // cumulative pairs with a differing donor
    int64_t accepted;        // cumulative accepted steps
    int32_t generation;      // generations completed
    int32_t best;            // best solution at the last finalize (lowest index on ties)
    int32_t new_elite;       // the last finalize replaced the elitist by solution `best`
    int32_t active;          // the last finalize closed a generation that ran
    int64_t start_tick;      // device wall clock at the start of a batch run
    int64_t done_tick;       // device wall clock when the elitist reached the target (or -1)
    uint64_t hash;           // accumulator of the state hash's gene and elitist terms
    uint64_t fi_fail;        // solutions the last generation's forced improvement replaced
                             // by the elitist
    uint32_t ls_any;         // local search: a flip happened in the current pass
    uint32_t stall;          // a dependency wait of the fused bit-sliced sweep gave up
    uint32_t fi_at[64];      // forced improvement of this generation: 0 while solution i has
                             // not improved, else kFiBase - t for the first class position t
                             // (in the generation's order) at which a step raised its fitness
    uint64_t ils_rej;        // iterated local search: solutions whose last round ended worse
                             // than they started (they return to P)
};

// A solution's forced improvement stops after the first class in which it improved, so a
// sweep at class position t skips solution i when fi_at[i] > kFiBase - t (it improved at an
// earlier position) and records an improvement by an atomic max of kFiBase - t: steps of
// the same class never see each other's records.
constexpr uint32_t kFiBase = 1u << 20;

// Accumulators that many blocks add into.  Device-scope atomics on one address serialise
// (tens of ns each), so every block adds into stripe (block index mod kStripes) and the
// finalize kernel sums the stripes.
constexpr int kStripes = 64;
struct alignas(64) Stripe {
    int64_t fit[64];         // fitness change per solution
    uint64_t evaluated;
    uint64_t accepted;
    uint64_t mism;           // solutions whose P differs from the elitist (vertex pass)
    uint64_t acc;            // solutions with an accepted GOM step in this generation
    uint64_t pad[4];
};

// Sweep modes: a GOM sweep, a GOM sweep that also records which solutions accepted a step
// (forced improvement on), and a forced-improvement sweep (the elitist as donor).
enum { kSweepGom = 0, kSweepGomTrack = 1, kSweepFi = 2 };

// One colour-class sweep launch.  Set records are stored in class order: class position p of
// class c is record s = class_start[c] + p, a block of int32 words at recs + roff[s] (layout
// described in gom_kernels.hip).
struct SweepArgs {
    const uint64_t *P;      // population at generation start, one word per vertex
    uint64_t *O;            // offspring, one word per vertex
    Stripe *stripes;
    const DevState *st;
    const int32_t *roff;    // record offsets (words), one per class position
    const int32_t *recs;    // record words
    int32_t rbase;          // first record word of the class
    int32_t rstride;        // words per record when the class's records are padded to one
                            // size, else 0 (then roff is used)
    uint64_t seed;
    int64_t target;         // generation runs only while elite_fitness < target
    int32_t N;              // population size
    int32_t gen;            // generation index g
    int32_t cls;            // colour class c
    int32_t cbase;          // first record of the class
    int32_t csize;          // number of sets in the class
    int32_t always;         // neutral rule: 1 = accept equal fitness always
    int32_t mode;           // kSweepGom, kSweepGomTrack or kSweepFi
    const uint64_t *E;      // elitist bits (forced improvement)
    int32_t coop;           // sets of kCoopMinMembers..kCoopMaxMembers members are left to
                            // the block-cooperative sweep (class launch, general FOS)
    int32_t n_large;        // block-cooperative sweep: number of such sets in the launch
    const int32_t *large_pos;  // ... and their class positions
    int32_t coop_cap;       // ... LDS words reserved per member array (the largest set)
    uint32_t *fi_at;        // DevState::fi_at of the state (forced improvement)
    int32_t fi_pos;         // forced-improvement sweep: class position in the order
    uint32_t *ls_any;       // DevState::ls_any of the state (local search)
    const int32_t *sw;      // bit-sliced sweep table (univariate FOS, degree <= 4): kSwRows
                            // arrays of sw_stride words, entry s = class position s
    int32_t sw_stride;
    // split sweep of the large sets of one group (few sets): one block per chunk of
    // kSplitMembers members, {slot, class position, first member, 0} per block, and per slot
    // (the set's index in the group) 64 donor masks, 64 fitness changes, 64 donor choices
    const int4 *smap;
    int32_t n_smap;
    uint64_t *split_D;
    int64_t *split_delta;
    int32_t *split_sel;
};

// Fused bit-sliced sweep: every colour class of a generation in one launch.  Block b owns
// chunk x = xcd_tile(b, grid) of every class (class c's positions are cut into `grid` chunks
// of clen[c] positions); it sweeps its chunk of each class in the generation's order and
// first waits until the chunks of earlier classes that hold a conflicting set (the same
// variable or a neighbour) are done in this launch.  A chunk is done when its flag holds the
// launch's epoch stamp (a host counter, so flags never need clearing).
constexpr int kFusedMaxGrid = 4096;
constexpr int kFusedMaxClasses = 8;
constexpr int kFusedMaxDepChunks = 32;  // widest dependency range (chunks) the fused sweep takes
constexpr uint32_t kFusedSpinLimit = 1u << 22;  // polls before a wait gives up (sets stall)
struct FusedArgs {
    SweepArgs a;
    const int4 *dep;   // [(c * grid + x) * k + c2]: two chunk ranges {lo0, hi0, lo1, hi1} of
                       // class c2 that chunk x of class c depends on ({0, -1}: unused)
    uint32_t *flags;   // [c * grid + x]: stamp of the last launch that finished the chunk
    uint32_t epoch;    // this launch's stamp
    int32_t k, grid;
    int32_t order[kFusedMaxClasses];   // class at each position of the generation's order
    int32_t cbase[kFusedMaxClasses];   // first class position (table entry) of class c
    int32_t csize[kFusedMaxClasses];
    int32_t clen[kFusedMaxClasses];    // chunk length of class c (positions)
};

// Groups of fewer than kSplitBelow large sets take the split sweep (three launches whose
// blocks each handle kSplitMembers members of one set) instead of one block per set.
constexpr int kSplitBelow = 128;
constexpr int kSplitMembers = 16;
// The split sweep's scratch: 64 donor masks, 64 fitness changes and 64 donor choices for each
// of kSplitBelow slots (the sets of one group), cleared at state initialization and left
// cleared by every sweep.
constexpr size_t kSplitScratchBytes =
    (size_t)kSplitBelow * 64 * (sizeof(uint64_t) + sizeof(int64_t) + sizeof(int32_t));

// The bit-sliced sweep's per-set table, one array per row so every load is coalesced: the
// variable u, its truth tables, its (up to 4) neighbours, then their edge weights.  A missing
// neighbour is u itself with weight 0.
enum { kSwU = 0, kSwTables = 1, kSwV = 2, kSwW = 6, kSwRows = 10 };

// Sets larger than the inline-member records are swept by a whole block (members split over
// its waves, a change mask and the offspring word of every member in LDS), up to the LDS
// capacity for those arrays; blocks of 256 threads up to kCoopSmallBlock members, else 1024.
constexpr int kCoopMinMembers = 15;
constexpr int kCoopMaxMembers = 8192;
constexpr int kCoopSmallBlock = 256;

// Generation end, in two launches: k_finalize (one block: fitness from the stripes, best
// solution, elitist decision, counters, generation count) then k_vertex_pass (all vertices:
// P <- O, elitist bits, solutions differing from the elitist into the stripes).
// One round's perturbation of the iterated local search (univariate FOS): solution i flips
// `flips` drawn variables in O, one after another.
struct PerturbArgs {
    const uint64_t *P;      // population planes (equal to O when the round starts; not written)
    uint64_t *O;            // offspring planes: the flips go here
    const int32_t *recs;    // set records; record of class position q at word roff[q]
    const int32_t *roff;
    Stripe *stripes;        // the flips' fitness changes go to stripe 0
    uint64_t seed;
    int32_t gen;            // generation count, first counter word of the draws
    int32_t round;          // round index r
    int32_t flips;          // flips per solution, 0..64
    int32_t n_sets;         // |F| (class positions 0..n_sets-1)
    int32_t N;
};

struct EpilogueArgs {
    uint64_t *P;
    uint64_t *O;            // offspring planes (read; rewritten when rows is set)
    const uint64_t *rows;   // if non-null: offspring as one bit row per solution (resident
                            // schedule); the vertex pass transposes them into P and O
    uint64_t *E;            // elitist bits, bit (v mod 64) of word v / 64
    int64_t *fit;
    DevState *st;
    Stripe *stripes;
    int64_t target;
    int32_t n;
    int32_t N;
    int32_t mode;           // 0: generation end, 1: initial elitist, 2: refresh flags only,
                            // 3: end of a local search (P <- O, elitist on strict
                            // improvement, no generation counted), 4: end of an iterated
                            // local search round (as 3, but a solution whose fitness fell
                            // keeps P)
    int32_t row_words;      // words per row, ceil(n / 64)
    int32_t fi;             // forced improvement on: replace the solutions that it did not
                            // improve by the elitist
};

enum { kEpiGeneration = 0, kEpiInit = 1, kEpiRefresh = 2, kEpiLocalSearch = 3, kEpiIterated = 4 };

// Resident schedule: one block per solution runs every colour class of a generation with
// the solution's offspring genes held in LDS (one byte per vertex), classes separated by
// block barriers.  Valid because donors are read from P (fixed during the generation) and
// the acceptance test only reads P_i's equality with the elitist, so solutions do not
// interact within a generation.
constexpr int kResidentThreads = 1024;
constexpr int kResidentMaxClasses = 1536;
constexpr int kResidentChunkSlots = kResidentThreads;  // Philox calls per round (8 sets each)

struct ResidentCtx {
    const uint64_t *P;
    uint64_t *rows;         // N rows of row_words words: bit (v mod 64) of word v / 64
    Stripe *stripes;
    const DevState *st;
    const int32_t *roff;
    const int32_t *recs;
    const int32_t *class_ptr;
    const int2 *class_rec;  // per class {first record word, record stride or 0}
    uint64_t seed;
    int64_t target;
    int32_t n;
    int32_t N;
    int32_t gen;            // generation index (single-state launches)
    int32_t k;
    int32_t always;
    int32_t row_words;
    int32_t fi;             // forced improvement after the classes
    const uint64_t *E;      // elitist bits
    uint32_t *fi_at;        // DevState::fi_at of the state
};

struct ResidentArgs {
    ResidentCtx c;
    uint16_t order[kResidentMaxClasses];  // class order of this generation
};

// Batch of independent instances run in lockstep: one launch per generation step for each of
// the sweep (one block per (instance, solution)), the finalize (one wave per instance) and the
// vertex pass (blocks of every instance's vertices).  Instances whose elitist has reached
// their target skip their work.
struct BatchInst {
    ResidentCtx res;
    EpilogueArgs epi;
    int32_t kind;           // 0 univariate records, 1 general
    int32_t order_fixed;    // class order ascending instead of shuffled
    int32_t vblock0;        // first vertex-pass block of the instance
    int32_t plds;           // the sweep keeps a copy of P in LDS
    int32_t bcl;            // swept by the batched class launches (offspring in the O planes)
    int32_t solo;           // too large for the resident schedule: the instance runs its own
                            // per-class sweeps and epilogue in each step (the batched
                            // finalize and vertex pass skip it)
};

// Dynamic LDS of the batched sweep before the resident part: class order and draws.
constexpr int kBatchOrderBytes = 4 * kResidentMaxClasses;

// Optional pair of events that a launch records with its own dispatch (start and end of the
// kernel's execution, as the profiler sees it); both null for a plain launch.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Bytes of the static arena (gom_state_init_static), one per device.
constexpr size_t kStaticArenaBytes = size_t(64) << 20;
// Device address of the current device's static arena (looked up once per device).
hipError_t static_arena_address(void **ptr);

// Batched class launch (FOS whose sets all have at most kBclMaxMembers members, in a batch):
// one launch per position t of the generation's class order covers class pi_i[t] of every
// such instance i.  Lane = solution (64 lanes per wave), so a set's record is read once for
// all solutions; a wave sweeps ppw consecutive positions (at most kBclPositions, the positions
// one Philox call serves), a block kBclWaves waves' worth (a tile).  Per step a planning pair
// of kernels draws every instance's class order and the prefix sums of its tiles per
// position.
constexpr int kBclWaves = 4;
constexpr int kBclPositions = 8;
constexpr int kBclThreads = 64 * kBclWaves;
constexpr int kBclMaxMembers = 9;  // largest set a class-launched batch instance may have
                                   // (neighbourhoods of degree 8)
constexpr int kBclMaxEntries = 72; // ... and most dependent edges of one of its sets
// Words past a record's start that a sweep may read (the record buffer's zero tail).
constexpr int kRecordTailWords = 192;
struct BclInst {
    const uint64_t *P;
    uint64_t *O;
    Stripe *stripes;
    const DevState *st;
    const int32_t *roff;
    const int32_t *recs;
    const int32_t *class_ptr;
    const int2 *class_rec;
    uint64_t seed;
    int64_t target;
    int32_t N, always, k, order_fixed;
    // univariate instance in the bit-sliced form: its bit-sliced table (one lane per set, all
    // solutions in one word, as k_uni_swar_sweep); uni = 0 for general records
    const int32_t *sw;
    int32_t sw_stride, uni, partition, pad;
};
// Blocks of the batched class-launch sweep for the current device (co-resident count).
hipError_t bcl_sweep_grid(int *grid);
struct BclPlan {
    const BclInst *insts;  // count instances
    uint16_t *order;       // [i * kmax + t]: class at position t of instance i's order
    int32_t *tiles;        // [t * (count + 1) + i]: tiles of instances before i at position t
    int32_t count, kmax, grid;
    int32_t ppw;           // consecutive class positions per wave (1..kBclPositions); a tile
                           // is kBclWaves * ppw positions
    // bit-sliced form (k_bcl_gs_sweep): lanes = slots (one or two a set, see gs_slots) over
    // all instances' classes at a position; `tiles` then holds slot prefix sums
    int32_t gs;            // 1: bit-sliced form
    int32_t gs_wb;         // its weight bits (7 or 13)
    int32_t gs_grid;       // blocks per launch (enough for every position's slots)
    uint64_t *nzm;         // [i]: solutions whose neutral steps are accepted (always, or those
                           // that differ from the elitist), written by k_bcl_order
    int4 *pos;             // [2 (t count + i) + 0/1]: instance i's class at position t as
                           // {class, first set, sets, generation}, {record start, stride, 0, 0},
                           // written by k_bcl_tiles in the bit-sliced form
};


// Kernel launchers (gom_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_init_population(uint64_t *P, uint64_t *O, int64_t *fit, DevState *st,
                                  Stripe *stripes, int n, int N, uint64_t seed, hipStream_t s);
hipError_t launch_zero_state(int64_t *fit, Stripe *stripes, hipStream_t s);
hipError_t launch_full_fitness(const uint64_t *P, const int32_t *eu, const int32_t *ev,
                               const int32_t *ew, int64_t m, int N, Stripe *stripes,
                               hipStream_t s);
// kind: 0 = univariate records, 1 = general records
// threads: block size, a multiple of 64 up to 512
// short_records: every record of the class has at most kShortRecordEntries entries (the
// one-set-per-wave sweep then fetches them 4 at a time).
constexpr int kShortRecordEntries = 16;
hipError_t launch_class_sweep(const SweepArgs &a, int kind, bool short_records, int max_grid,
                              int threads, hipStream_t s, KernelEvents ev = {});
// Class sweep of small general sets (at most kBclMaxMembers members, kBclMaxEntries dependent
// edges, population above 32) with each set staged by its wave in two rounds of loads.
hipError_t launch_class_sweep_staged(const SweepArgs &a, int max_grid, int threads,
                                     hipStream_t s, KernelEvents ev = {});
// Bit-parallel class sweep: univariate FOS, degree <= 4, per-set |weight| sums below 2^30.
// Block-cooperative sweep of the large sets of one class (a.n_large blocks); max_members:
// the largest of them (dynamic LDS of 8 bytes per member).
hipError_t launch_split_sweep(const SweepArgs &a, hipStream_t s);
// One colour class of the local search (univariate FOS records).
hipError_t launch_ls_sweep(const SweepArgs &a, int max_grid, hipStream_t s);
hipError_t launch_perturb(const PerturbArgs &a, hipStream_t s);
hipError_t launch_large_set_sweep(const SweepArgs &a, int max_members, int threads,
                                  hipStream_t s);
// narrow: the host has checked that a block's per-solution fitness sums fit in int32.
hipError_t launch_uni_swar_sweep(const SweepArgs &a, bool partition, bool narrow, int max_grid,
                                 hipStream_t s, KernelEvents ev = {});
constexpr int kSwarThreads = 256;  // threads per block of the bit-sliced sweep
// Bit-sliced sweep of small general sets (lane = set): classes whose sets have at most
// kGsMaxMembers members, whose per-set sum of |w| over the dependent edges is at most
// kGsMaxWeightSum (the bit-sliced sum 2 W stays below 2^15) and whose largest |w| has at most
// kGsMaxWeightBits bits (the host also requires a least class size).
constexpr int kGsThreads = 256;
constexpr int kGsEntryBatch = 8;   // dependent-edge entries whose loads are issued together
constexpr int kGsEntryBatchBcl = 8;   // ... in the batched class launches
constexpr int kGsMaxMembers = 9;
constexpr int64_t kGsMaxWeightSum = 16383;
constexpr int kGsMaxWeightBits = 13;
// Lane slots of a class of `csize` sets under the bit-sliced general sweep (a multiple of
// 16): 16 slots hold 8 positions x 2 halves (population above 32) or 16 positions.
__host__ __device__ __forceinline__ int gs_slots(int csize, int halves) {
    const int per = 16 / halves;  // positions per 16 slots
    return (csize + per - 1) / per * 16;
}
// ... in the batched class launches, where each half is split between kGsPartsBcl lanes: 8
// positions take 8 x parts x halves slots; the count is rounded up to a wave (64) so that every
// instance's slots start at a multiple of 64 and a lane's partners (8, 16, ... lanes away) are
// always in its wave.
constexpr int kGsPartsBcl = 4;
__host__ __device__ __forceinline__ int gs_slots_bcl(int csize, int halves) {
    const int n = (csize + 7) / 8 * 8 * kGsPartsBcl * halves;
    return (n + 63) / 64 * 64;
}
// ... and of a univariate instance's class (one lane a set), also rounded to a wave.
__host__ __device__ __forceinline__ int gs_slots_uni(int csize) { return (csize + 63) / 64 * 64; }
hipError_t launch_gen_swar_sweep(const SweepArgs &a, int members, int weight_bits, int max_grid,
                                 hipStream_t s, KernelEvents ev);
// Fused form (one cooperative launch per generation; see FusedArgs).
hipError_t launch_uni_swar_fused(const FusedArgs &f, bool partition, bool narrow,
                                 hipStream_t s);
// Blocks of the fused sweep that the current device holds at once (its grid), or an error.
hipError_t fused_swar_grid(int *grid);
// plds: keep a copy of P in LDS (needs resident_lds_bytes(n, true) of LDS).
hipError_t launch_resident_sweep(const ResidentArgs &a, int kind, bool plds, hipStream_t s,
                                 KernelEvents ev = {});
// Batched generation step over `count` instances.  The sweep runs as one launch per group of
// blocks (blk[first .. first + count) = {instance, solution}) with `threads` threads (256 or
// 1024) and `lds` dynamic LDS bytes per block; then the finalize (one wave per instance) and
// the vertex pass (vblocks blocks, vblk[b] = instance).  ev: optional events, the start
// recorded by the first sweep launch and the stop by the last.
struct BatchLaunch {
    int first, count, threads, kind;  // kind: FOS kind of the group's instances
    size_t lds;
};
// Blocks of the batched sweep (threads = 256 or 1024, FOS kind) that a CU holds at once by
// registers and threads alone (without dynamic LDS).
hipError_t batch_sweep_occupancy(int threads, int kind, int *blocks);
// Allows each group's k_batch_sweep blocks their dynamic LDS (once per size; not a stream
// operation, so it is done before a step is captured into a graph).
hipError_t prepare_batch_step(const BatchLaunch *groups, int n_groups);
hipError_t launch_batch_step(const BatchInst *insts, int count, const int2 *blk,
                             const BatchLaunch *groups, int n_groups, const int32_t *vblk,
                             int vblocks, const BclPlan &bcl, hipStream_t s,
                             KernelEvents ev = {});
hipError_t launch_batch_mark(const BatchInst *insts, int count, hipStream_t s);
// Pack every instance's DevState into out[count].
hipError_t launch_batch_gather(const BatchInst *insts, int count, DevState *out, hipStream_t s);
// State hash, gene and elitist terms: st->hash <- sum over v of the terms of bit i of X[v] at
// byte position i*n + v (every solution i < N) and of the elitist bit v at position ebase + v.
hipError_t launch_state_hash(const uint64_t *X, const uint64_t *E, int n, int N, uint64_t ebase,
                             DevState *st, hipStream_t s);
// Generation end: finalize (one block) then the vertex pass.
hipError_t launch_epilogue(const EpilogueArgs &a, hipStream_t s);
// Dynamic LDS bytes of the resident sweep for n vertices, with or without the P copy.
size_t resident_lds_bytes(int n, bool plds, int threads = kResidentThreads);

}  // namespace gom
