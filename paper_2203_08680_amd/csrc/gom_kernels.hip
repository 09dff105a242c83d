// gom_kernels.hip -- CDNA4 (gfx950) kernels of libgom.
//
// Data layout in HBM (one state):
//   P, O   population at generation start and offspring, one 64-bit word per vertex; bit i of
//          word v is gene v of solution i (bit-planes: a vertex's genes for the whole
//          population, up to 64 solutions, travel in one 8-byte access).
//   E      elitist genes, bit (v mod 64) of word v / 64.
//   fit    int64 fitness per solution; stripes: per-block accumulators (see Stripe).
//   records of the FOS sets in colour-class order (layout below).
//
// A generation runs under one of three schedules with identical results:
//   class launch: one k_class_sweep launch per colour class (in the generation's class
//     order), lane = solution, offspring in the O planes; a class's sets of 15 to 8192
//     members go to the split sweep (k_split_donors, k_split_delta, k_split_commit: blocks
//     of 16-member chunks) when the class holds fewer than 128 of them, else to
//     k_large_set_sweep (one block per set);
//   bit-sliced:   one k_uni_swar_sweep launch per colour class, lane = set, all solutions of
//     the set in one word (univariate FOS, degree <= 4);
//   resident:     one k_resident_sweep launch (block = solution, offspring in LDS, all
//     classes), offspring written back as one bit row per solution;
// then k_finalize (one block) and k_vertex_pass (P <- O, elitist, equality flags).  Also:
// k_batch_* (many instances in lockstep), k_ls_sweep (the colouring-parallel local search),
// k_perturb (its iterated form's perturbation), k_state_hash.  Integer arithmetic only, so every result is exact and independent of the
// order in which waves run.
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>

#include "gom_internal.h"

namespace gom {
namespace {

static_assert(kStripes == 64, "one stripe per lane of a wave");

constexpr int kSweepMaxThreads = 512;  // class sweep blocks: 64 to 512 threads
constexpr int kEpiThreads = 256;
constexpr int kFitThreads = 256;

__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t bit_of(uint64_t w, uint32_t i) {
    return (uint32_t)(w >> i) & 1u;
}

// Index of the r-th (0-based) set bit of x; requires r < popcount(x).
__device__ __forceinline__ uint32_t select_bit(uint64_t x, uint32_t r) {
    uint32_t base = 0;
    uint32_t w = (uint32_t)x;
    uint32_t c = (uint32_t)__popc(w);
    if (r >= c) { r -= c; w = (uint32_t)(x >> 32); base = 32; }
    c = (uint32_t)__popc(w & 0xFFFFu);
    if (r >= c) { r -= c; w >>= 16; base += 16; }
    c = (uint32_t)__popc(w & 0xFFu);
    if (r >= c) { r -= c; w >>= 8; base += 8; }
    c = (uint32_t)__popc(w & 0xFu);
    if (r >= c) { r -= c; w >>= 4; base += 4; }
    c = (uint32_t)__popc(w & 0x3u);
    if (r >= c) { r -= c; w >>= 2; base += 2; }
    if (r >= (w & 1u)) base += 1;
    return base;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD b mod 8), and each
// XCD has its own L2.  xcd_tile maps block b to a logical tile so that every XCD works on one
// contiguous range of tiles: neighbouring sets share population words, which are then
// fetched into one L2 instead of several.  A bijection on [0, G).
__device__ __forceinline__ int xcd_tile(int b, int G) {
    constexpr int kXcds = 8;
    const int x = b % kXcds, q = b / kXcds;
    const int per = G / kXcds, rem = G % kXcds;
    return x * per + (x < rem ? x : rem) + q;
}

// Wave reductions with a wave-uniform result.  Each of the four 16-lane rows is reduced by
// DPP rotations of 1, 2, 4 and 8 lanes (after step k every lane holds its row's 2^k-lane
// cyclic window, so after the fourth step the whole row, each lane counted once); the rows'
// results are then read from lanes 0, 16, 32 and 48.  Every lane of the wave must be active.
constexpr int kDppRor1 = 0x121, kDppRor2 = 0x122, kDppRor4 = 0x124, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t read_lane(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

__device__ __forceinline__ uint32_t row_or32(uint32_t x) {
    x |= dpp_u32<kDppRor1>(x);
    x |= dpp_u32<kDppRor2>(x);
    x |= dpp_u32<kDppRor4>(x);
    x |= dpp_u32<kDppRor8>(x);
    return x;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
    const uint32_t lo = row_or32((uint32_t)x), hi = row_or32((uint32_t)(x >> 32));
    const uint32_t l = read_lane(lo, 0) | read_lane(lo, 16) | read_lane(lo, 32) | read_lane(lo, 48);
    const uint32_t h = read_lane(hi, 0) | read_lane(hi, 16) | read_lane(hi, 32) | read_lane(hi, 48);
    return ((uint64_t)h << 32) | l;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
    x += dpp_u32<kDppRor1>(x);
    x += dpp_u32<kDppRor2>(x);
    x += dpp_u32<kDppRor4>(x);
    x += dpp_u32<kDppRor8>(x);
    return read_lane(x, 0) + read_lane(x, 16) + read_lane(x, 32) + read_lane(x, 48);
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    return ((uint64_t)dpp_u32<CTRL>((uint32_t)(x >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)x);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
    uint64_t x = (uint64_t)v;  // two's complement: the sum modulo 2^64 is the int64 sum
    x += dpp_u64<kDppRor1>(x);
    x += dpp_u64<kDppRor2>(x);
    x += dpp_u64<kDppRor4>(x);
    x += dpp_u64<kDppRor8>(x);
    uint64_t s = 0;
#pragma unroll
    for (int r = 0; r < 64; r += 16)
        s += ((uint64_t)read_lane((uint32_t)(x >> 32), r) << 32) | read_lane((uint32_t)x, r);
    return (int64_t)s;
}

// Solutions (bit i) whose forced improvement raised their fitness at a class position before
// pos in this generation (lane i reads solution i's record; every lane must be active).
__device__ __forceinline__ uint64_t fi_done_before(const uint32_t *fi_at, int pos) {
    return ballot64(fi_at[threadIdx.x & 63] > kFiBase - (uint32_t)pos);
}

// ------------------------------------------------------------------------------------------
// Initial population (Algorithm 3, InitializePopulation): gene v of solution i is bit
// (v mod 32) of word ((v / 32) mod 4) of Philox(seed; kInitStream, i, v / 128, 0).
// One wave per 128 vertices: lane i draws solution i's 128 genes, then 128 ballots turn them
// into the 128 population words, two per lane, stored coalesced.  Block 0 also clears the
// fitness, the stripes and the run scalars.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_population(uint64_t *P, uint64_t *O, int64_t *fit,
                                                         DevState *st, Stripe *stripes, int n,
                                                         int N, uint64_t seed) {
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) fit[threadIdx.x] = 0;
        uint64_t *sw = reinterpret_cast<uint64_t *>(stripes);
        for (int q = threadIdx.x; q < kStripes * (int)(sizeof(Stripe) / 8); q += 256) sw[q] = 0;
        if (threadIdx.x == 0) {
            st->elite_fitness = INT64_MIN;
            st->evaluated = 0;
            st->accepted = 0;
            st->generation = 0;
            st->best = 0;
            st->new_elite = 0;
            st->active = 0;
            st->start_tick = 0;
            st->done_tick = -1;
            st->stall = 0;
        }
    }
    const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk * 128 >= n) return;
    U32x4 r = {0u, 0u, 0u, 0u};
    if (lane < N) r = philox(seed, kInitStream, (uint32_t)lane, (uint32_t)blk, 0u);
    const uint32_t words[4] = {r.x, r.y, r.z, r.w};
    uint64_t w0 = 0, w1 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int b = 0; b < 32; ++b) {
            const uint64_t m = ballot64(lane < N && ((words[q] >> b) & 1u));
            const int t = q * 32 + b;
            if ((t & 63) == lane) {
                if (t < 64) w0 = m; else w1 = m;
            }
        }
    }
    const int v0 = blk * 128 + lane, v1 = v0 + 64;
    if (v0 < n) { P[v0] = w0; O[v0] = w0; }
    if (v1 < n) { P[v1] = w1; O[v1] = w1; }
}

__global__ __launch_bounds__(256) void k_zero_state(int64_t *fit, Stripe *stripes) {
    if (threadIdx.x < 64) fit[threadIdx.x] = 0;
    uint64_t *sw = reinterpret_cast<uint64_t *>(stripes);
    for (int q = threadIdx.x; q < kStripes * (int)(sizeof(Stripe) / 8); q += 256) sw[q] = 0;
}

// ------------------------------------------------------------------------------------------
// Full Max-Cut fitness of every solution (Section 6.2): one wave per edge at a time, lane i
// adds the weight when bit i of P[u] xor P[v] is set (the edge is cut in solution i).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kFitThreads) void k_full_fitness(const uint64_t *P,
                                                              const int32_t *eu,
                                                              const int32_t *ev,
                                                              const int32_t *ew, int64_t m,
                                                              int N, Stripe *stripes) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * (kFitThreads / 64);
    for (int64_t e = (int64_t)blockIdx.x * (kFitThreads / 64) + wave; e < m; e += stride) {
        const uint64_t x = P[eu[e]] ^ P[ev[e]];
        if (bit_of(x, (uint32_t)lane)) acc += ew[e];
    }
    __shared__ int64_t red[kFitThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && (int)threadIdx.x < N) {
        int64_t s = 0;
#pragma unroll
        for (int w = 0; w < kFitThreads / 64; ++w) s += red[w * 64 + threadIdx.x];
        if (s)
            atomicAdd((unsigned long long *)&stripes[blockIdx.x % kStripes].fit[threadIdx.x],
                      (unsigned long long)s);
    }
}

// ------------------------------------------------------------------------------------------
// Set records (built on the host in colour-class order, one per class position s, starting
// at word roff[s] on a 16-byte boundary):
//   univariate FOS:  [u, nd, tables, 0] then nd entries {v, w}: the neighbours of the set's
//                    variable u and the edge weights; for nd <= 4, `tables` holds the
//                    bit-sliced sweep's truth tables (low 16 bits: flip gain > 0, high 16
//                    bits: gain == 0, bit p for the pattern p of same-gene far ends)
//   small set (nm <= 14 variables, n < 2^27): [nm, nd, u_0..u_13] then nd entries {x, w}
//                    (unused member slots hold -1); x holds the position a of the entry's
//                    own endpoint in bits 27..30, and either the outside neighbour v (bit 31
//                    clear) or, for an edge inside the set (listed once, under its lower
//                    position), the other endpoint's position b (bit 31 set) in bits 0..26
//   large set:       [nm, nd, 0 x 14] then u_0..u_{nm-1}, end_0..end_{nm-1}, then from the
//                    next 16-byte boundary nd entries {x, w} with x = v (outside) or ~b
//                    (inside, b > a)
// The partial evaluation of Section 2.2 / Algorithm 4 reads exactly these entries: the
// subfunctions (edges) that depend on a variable of the set.
// ------------------------------------------------------------------------------------------
constexpr int kSmallSet = 14;
constexpr int kSmallPosShift = 27;
constexpr uint32_t kSmallIdx = (1u << kSmallPosShift) - 1u;
constexpr int kBatch = 8;  // entries fetched together

struct PairOut {
    uint32_t cnt;    // eligible donors
    bool acc;        // step accepted
    int64_t delta;   // fitness change of the step
};

// Donor words for forced improvement: every "solution" carries the elitist's gene, so the
// donor mask is all ones where the elitist differs from O_i and the chosen donor is the
// elitist.
struct EliteWords {
    const uint64_t *E;
    __device__ __forceinline__ uint64_t operator[](int v) const {
        return 0ull - ((E[v >> 6] >> (v & 63)) & 1ull);
    }
};

// Solutions set in a wave's per-lane flag (lane = group * G + solution).
template <int G>
__device__ __forceinline__ uint64_t solution_mask(bool flag) {
    uint64_t m = ballot64(flag);
    if constexpr (G < 64) {
#pragma unroll
        for (int g = 1; g < 64 / G; ++g) m |= m >> (g * G);
        m &= (1ull << G) - 1ull;
    }
    return m;
}

// A load through the constant address space.  With a wave-uniform address the backend turns
// it into a scalar load (into SGPRs, through the scalar cache, no lane broadcast).  Only for
// memory that no kernel writes while another reads it (the set records).
template <class T>
__device__ __forceinline__ T const_load(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}
__device__ __forceinline__ int4 const_load(const int4 *p) {
    const int32_t *q = reinterpret_cast<const int32_t *>(p);
    return make_int4(const_load(q), const_load(q + 1), const_load(q + 2), const_load(q + 3));
}
__device__ __forceinline__ int2 const_load(const int2 *p) {
    const int32_t *q = reinterpret_cast<const int32_t *>(p);
    return make_int2(const_load(q), const_load(q + 1));
}

// Offspring bits of solution i in the O planes (class-launch schedule).
struct PlaneBits {
    static constexpr bool kLocal = false;  // reads go to global memory
    const uint64_t *O;
    uint32_t i;
    __device__ __forceinline__ uint32_t operator()(int v) const { return bit_of(O[v], i); }
};

// Offspring bits of one solution in LDS, one byte per vertex (resident schedule).
struct LdsBits {
    static constexpr bool kLocal = true;   // reads go to LDS: cheap to repeat
    const uint8_t *ob;
    __device__ __forceinline__ uint32_t operator()(int v) const { return ob[v]; }
};

__device__ __forceinline__ int32_t signed_w(uint32_t same, int32_t w) { return same ? w : -w; }

// GOM step (Algorithm 2) of solution i on the set whose record starts at R.  `bits` reads
// O_i; `commit(u, flip)` is called once per member u (by every lane of a group, so it may
// use cross-lane operations) and flips O_i[u] when `flip`.  `h` is the 16-bit donor draw,
// `cand` the mask of possible donors (every solution but i).
// The first words of a record: the header and the first entry batches (8 entries for a
// univariate record, 16 for a small set), fetched together so a kernel can issue them before
// it waits for anything else.  Reads past a short record stay inside the buffer's zero tail;
// entries beyond nd are masked before use.
// A record's first words: header, then two batches of B entries.
template <int B>
struct HeadT {
    int4 h0, h1, h2, h3;
    int2 en0[B], en1[B];
};
using Head = HeadT<kBatch>;

// Record reader: a record's words are consecutive, read with vector loads.
struct AosRec {
    const int32_t *R;
    __device__ __forceinline__ int32_t w(int k) const { return R[k]; }
    __device__ __forceinline__ int4 q(int k) const {
        return reinterpret_cast<const int4 *>(R)[k];
    }
    __device__ __forceinline__ int2 e(int base, int t) const {
        return reinterpret_cast<const int2 *>(R + base)[t];
    }
};

// Reader for a record that every lane of the wave reads (class launch with one set per wave):
// the record address is wave-uniform, so its words are scalar loads and its decoding runs on
// the scalar unit.
struct UniformAosRec {
    const int32_t *R;
    __device__ __forceinline__ int32_t w(int k) const { return const_load(R + k); }
    __device__ __forceinline__ int4 q(int k) const {
        return const_load(reinterpret_cast<const int4 *>(R) + k);
    }
    __device__ __forceinline__ int2 e(int base, int t) const {
        return const_load(reinterpret_cast<const int2 *>(R + base) + t);
    }
};

template <int KIND, int B = kBatch, class Rec>
__device__ __forceinline__ HeadT<B> load_head(const Rec &R) {
    HeadT<B> hd;
    hd.h0 = R.q(0);
    if constexpr (KIND == 0) {
#pragma unroll
        for (int t = 0; t < B; ++t) hd.en0[t] = R.e(4, t);
    } else {
        hd.h1 = R.q(1);
        hd.h2 = R.q(2);
        hd.h3 = R.q(3);
#pragma unroll
        for (int t = 0; t < B; ++t) {
            hd.en0[t] = R.e(16, t);
            hd.en1[t] = R.e(16, B + t);
        }
    }
    return hd;
}

// Change of one dependent edge of a small-set record (entry e of nd): x holds the member
// position a of its own end, and the outside vertex v (bit 31 clear) or the inside end's
// position b; ovx is O_i at the outside end.  om / cm: O_i bits / changed members by position.
__device__ __forceinline__ int64_t small_edge(int e, int nd, int2 en, uint32_t ovx, uint32_t om,
                                              uint32_t cm) {
    const int x = e < nd ? en.x : (int)0x80000000;  // past nd: a = b = 0, no flip
    const uint32_t a = ((uint32_t)x >> kSmallPosShift) & 15u;
    const uint32_t y = (uint32_t)x & kSmallIdx;
    const uint32_t oa = (om >> a) & 1u, ca = (cm >> a) & 1u;
    const bool inside = x < 0;
    const uint32_t ov = inside ? (om >> y) & 1u : ovx;
    const uint32_t flip = inside ? ca ^ ((cm >> y) & 1u) : ca;
    return flip ? signed_w(oa == ov, en.y) : 0;
}

// GOM step on a small set (at most M member slots, M >= nm) with the offspring in the O
// planes (class launch).  Every word the step needs is loaded before the first is used, so
// the loads are in flight together: the population and offspring words of the member slots
// (a slot past nm reads the first member again and is masked out) and the offspring words at
// the far ends of the first two entry batches (entries past nd read vertex 0).  The commit
// writes each changed member's new word from the word already loaded.
template <int M, int B, class Rec, class Words, class Commit>
__device__ __forceinline__ PairOut small_pair_planes(const Rec &R, const HeadT<B> &hd, const Words &P,
                                                     const PlaneBits &bits, Commit commit,
                                                     uint64_t cand, uint32_t h, bool neutral_ok) {
    PairOut out{0u, false, 0};
    const int4 h0 = hd.h0, h1 = hd.h1, h2 = hd.h2, h3 = hd.h3;
    const int nm = h0.x, nd = h0.y;
    const int mem[kSmallSet] = {h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x,
                                h2.y, h2.z, h2.w, h3.x, h3.y, h3.z, h3.w};
    auto far_index = [&](int e, int2 en) {
        return (int)((uint32_t)(e < nd ? en.x : 0) & kSmallIdx);
    };
    uint64_t pw[M], ow[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int u = k < nm ? mem[k] : mem[0];
        pw[k] = P[u];
        ow[k] = bits.O[u];
    }
    uint32_t ov0[B], ov1[B];
#pragma unroll
    for (int t = 0; t < B; ++t) {
        ov0[t] = bits(far_index(t, hd.en0[t]));
        ov1[t] = bits(far_index(B + t, hd.en1[t]));
    }
    uint32_t om = 0;
    uint64_t D = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint32_t ok = bit_of(ow[k], bits.i);
        const uint64_t diff = pw[k] ^ (0ull - (uint64_t)ok);
        om |= (k < nm ? ok : 0u) << k;
        D |= k < nm ? diff : 0ull;
    }
    D &= cand;
    out.cnt = (uint32_t)__popcll(D);
    const uint32_t d = out.cnt ? select_bit(D, (h * out.cnt) >> 16) : 0u;
    uint32_t cm = 0;
#pragma unroll
    for (int k = 0; k < M; ++k)
        cm |= (k < nm ? bit_of(pw[k], d) ^ ((om >> k) & 1u) : 0u) << k;
    int64_t delta = 0;
#pragma unroll
    for (int t = 0; t < B; ++t) {
        delta += small_edge(t, nd, hd.en0[t], ov0[t], om, cm);
        delta += small_edge(B + t, nd, hd.en1[t], ov1[t], om, cm);
    }
    for (int e0 = 2 * B; e0 < nd; e0 += B) {
        int2 en[B];
        uint32_t ov[B];
#pragma unroll
        for (int t = 0; t < B; ++t) en[t] = R.e(16, e0 + t);
#pragma unroll
        for (int t = 0; t < B; ++t) ov[t] = bits(far_index(e0 + t, en[t]));
#pragma unroll
        for (int t = 0; t < B; ++t) delta += small_edge(e0 + t, nd, en[t], ov[t], om, cm);
    }
    out.delta = delta;
    out.acc = out.cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (k < nm) commit.store(mem[k], out.acc && ((cm >> k) & 1u), ow[k]);
    return out;
}

template <int KIND, int B, class Rec, class Words, class Bits, class Commit>
__device__ __forceinline__ PairOut gom_pair(const Rec &R, const HeadT<B> &hd, const Words &P,
                                            Bits bits, Commit commit, uint64_t cand, uint32_t h,
                                            bool neutral_ok) {
    PairOut out{0u, false, 0};
    const int4 h0 = hd.h0;
    if constexpr (KIND == 0) {
        // one variable u: the donor always differs at u, so C = {u} whenever a donor exists
        int2 en[B];
#pragma unroll
        for (int t = 0; t < B; ++t) en[t] = hd.en0[t];
        const int u = h0.x, nd = h0.y;
        const uint32_t ou = bits(u);
        const uint64_t D = (P[u] ^ (0ull - (uint64_t)ou)) & cand;
        out.cnt = (uint32_t)__popcll(D);
        int64_t delta = 0;
        for (int e0 = 0; e0 < nd; e0 += B) {
            if (e0 > 0) {
#pragma unroll
                for (int t = 0; t < B; ++t) en[t] = R.e(4, e0 + t);
            }
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const bool ok = e0 + t < nd;
                const int v = ok ? en[t].x : u;
                delta += ok ? signed_w(ou == bits(v), en[t].y) : 0;
            }
        }
        out.delta = delta;
        out.acc = out.cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
        commit(u, out.acc);
        return out;
    } else {
        const int nm = h0.x, nd = h0.y;
        if (nm <= kSmallSet) {
            if constexpr (!Bits::kLocal) {
                // class launch: sets of up to 4 and 5 members (neighbourhoods of degree 3 and
                // 4, the torus's) load 4 and 5 member slots, up to 8 members 8, larger ones all
                // 14
                if (nm <= 4)
                    return small_pair_planes<4>(R, hd, P, bits, commit, cand, h, neutral_ok);
                if (nm <= 5)
                    return small_pair_planes<5>(R, hd, P, bits, commit, cand, h, neutral_ok);
                if (nm <= 8)
                    return small_pair_planes<8>(R, hd, P, bits, commit, cand, h, neutral_ok);
                return small_pair_planes<kSmallSet>(R, hd, P, bits, commit, cand, h,
                                                    neutral_ok);
            } else {
            // resident schedule: bits in LDS, read again where they are needed instead of
            // being held in registers (1024-thread blocks have 128 registers per lane).
            // Entries past nd belong to the next record and read vertex 0 instead; an inside
            // entry's b is below nm <= n, so every index is a vertex and no load needs a branch
            const int4 h1 = hd.h1, h2 = hd.h2, h3 = hd.h3;
            const int mem[kSmallSet] = {h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x,
                                        h2.y, h2.z, h2.w, h3.x, h3.y, h3.z, h3.w};
            auto far_end = [&](int e, int2 en) {
                return bits((int)((uint32_t)(e < nd ? en.x : 0) & kSmallIdx));
            };
            uint32_t om = 0;
            uint64_t D = 0;
#pragma unroll
            for (int k = 0; k < kSmallSet; ++k) {
                if (k < nm) {
                    const uint64_t w = P[mem[k]];
                    const uint32_t ok = bits(mem[k]);
                    om |= ok << k;
                    D |= w ^ (0ull - (uint64_t)ok);
                }
            }
            D &= cand;
            out.cnt = (uint32_t)__popcll(D);
            const uint32_t d = out.cnt ? select_bit(D, (h * out.cnt) >> 16) : 0u;
            uint32_t cm = 0;
#pragma unroll
            for (int k = 0; k < kSmallSet; ++k)
                if (k < nm) cm |= (bit_of(P[mem[k]], d) ^ ((om >> k) & 1u)) << k;
            int64_t delta = 0;
#pragma unroll
            for (int t = 0; t < B; ++t) {
                delta += small_edge(t, nd, hd.en0[t], far_end(t, hd.en0[t]), om, cm);
                delta += small_edge(B + t, nd, hd.en1[t], far_end(B + t, hd.en1[t]),
                                    om, cm);
            }
            // further entries a batch at a time: the batch's loads, then its far-end bits
            for (int e0 = 2 * B; e0 < nd; e0 += B) {
                int2 en[B];
                uint32_t ov[B];
#pragma unroll
                for (int t = 0; t < B; ++t) en[t] = R.e(16, e0 + t);
#pragma unroll
                for (int t = 0; t < B; ++t) ov[t] = far_end(e0 + t, en[t]);
#pragma unroll
                for (int t = 0; t < B; ++t)
                    delta += small_edge(e0 + t, nd, en[t], ov[t], om, cm);
            }
            out.delta = delta;
            out.acc = out.cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
#pragma unroll
            for (int k = 0; k < kSmallSet; ++k)
                if (k < nm) commit(mem[k], out.acc && ((cm >> k) & 1u));
            return out;
            }
        } else {
            // members at words 16.., their entry ends at 16 + nm.., entries from the next
            // 4-word boundary
            const int eb = (16 + 2 * nm + 3) & ~3;
            uint64_t D = 0;
            for (int k = 0; k < nm; ++k) {
                const int u = R.w(16 + k);
                D |= P[u] ^ (0ull - (uint64_t)bits(u));
            }
            D &= cand;
            out.cnt = (uint32_t)__popcll(D);
            const uint32_t d = out.cnt ? select_bit(D, (h * out.cnt) >> 16) : 0u;
            int64_t delta = 0;
            int e = 0;
            for (int k = 0; k < nm; ++k) {
                const int u = R.w(16 + k);
                const uint32_t ou = bits(u);
                const uint32_t cu = bit_of(P[u], d) ^ ou;
                for (const int e1 = R.w(16 + nm + k); e < e1; ++e) {
                    const int2 en = R.e(eb, e);
                    uint32_t ov, flip;
                    if (en.x >= 0) {
                        ov = bits(en.x);
                        flip = cu;
                    } else {
                        const int vb = R.w(16 + ~en.x);
                        ov = bits(vb);
                        flip = cu ^ (bit_of(P[vb], d) ^ ov);
                    }
                    delta += flip ? signed_w(ou == ov, en.y) : 0;
                }
            }
            out.delta = delta;
            out.acc = out.cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
            for (int k = 0; k < nm; ++k) {
                const int u = R.w(16 + k);
                const uint32_t cu = bit_of(P[u], d) ^ bits(u);
                commit(u, out.acc && cu);
            }
            return out;
        }
    }
}

// ------------------------------------------------------------------------------------------
// One colour class of one generation (Algorithm 3, the body of the loop over groups; the GOM
// step of Algorithm 2 for every (solution, set) pair of the class at once).
//
// Mapping: a group of G lanes (G = 16, 32 or 64, the population rounded up) takes one set of
// the class; lane i of the group is solution i.  Waves work independently (no block
// barriers): wave w takes class positions w * 64/G .. + 64/G - 1, then strides by the number
// of waves in the grid.  All sets of one class are independent (no shared or adjacent
// variables), so groups never read a word that another group of the same launch writes, and
// each O word of a set is written by exactly one lane.
//
// Per pair (solution i, set F_j at class position p):
//   D      = solutions d != i whose P genes differ from O_i somewhere on F_j (64-bit mask,
//            OR over the members of (P[u] xor broadcast(O_i[u])))
//   h      = 16-bit field (p mod 8) of Philox(seed; g, c, i, p / 8), drawn by the lane
//   donor  = the r-th set bit of D with r = (h * |D|) >> 16
//   C      = members u where the donor's gene differs from O_i[u]
//   delta  = sum over the set's dependent edges of the change of the cut: an outside edge
//            (u, v) changes when u is in C, an inside edge when exactly one end is in C; the
//            change is +w if the edge was uncut, -w if it was cut
//   accept = |D| > 0 and (delta > 0 or (delta == 0 and (always or P_i != elitist)))
//   commit = one word store per member: O[u] ^= ballot(accept and u in C)
// Fitness changes and counts are summed per wave and added to the wave's stripe.
// ------------------------------------------------------------------------------------------
template <int G>
struct PlaneCommit {
    uint64_t *O;
    int grp;
    uint32_t i;
    __device__ __forceinline__ void operator()(int u, bool flip) const {
        uint64_t fm = ballot64(flip);
        if constexpr (G < 64) fm = (fm >> (grp * G)) & ((1ull << G) - 1ull);
        if (fm != 0 && i == 0) O[u] ^= fm;
    }
    // the same from the word the group already loaded: no other group writes u in this class
    __device__ __forceinline__ void store(int u, bool flip, uint64_t old) const {
        uint64_t fm = ballot64(flip);
        if constexpr (G < 64) fm = (fm >> (grp * G)) & ((1ull << G) - 1ull);
        if (fm != 0 && i == 0) O[u] = old ^ fm;
    }
};

// B: record entries fetched per batch (4 for classes whose records have at most 16 entries:
// fewer scalar registers live, fewer spills; else 8).
// PPW: class positions per group and wave tile, 1 or 8.  With 8, a group sweeps the eight
// consecutive positions whose donor draws come from one Philox call, and draws it once
// instead of once per position (used for classes large enough that every group strides over
// at least eight positions anyway).
template <int G, int KIND, bool FI, int B, int PPW = 1>
__global__ __launch_bounds__(kSweepMaxThreads) void k_class_sweep(SweepArgs a) {
    static_assert(PPW == 1 || (PPW == 8 && KIND != 0 && !FI), "shared draws: general, GOM");
    constexpr int GPW = 64 / G;          // sets per wave
    const int lane = threadIdx.x & 63;
    const int grp = lane / G;
    const uint32_t i = (uint32_t)(lane % G);
    const int wpb = (int)(blockDim.x >> 6);                        // waves per block
    const int gw = xcd_tile((int)blockIdx.x, (int)gridDim.x) * wpb +
                   (int)(threadIdx.x >> 6);                        // global wave (tile order)
    const int nwaves = gridDim.x * wpb;
    // one set per wave (G = 64): the record is wave-uniform (scalar loads); with several sets
    // per wave it is read with per-lane vector loads
    constexpr bool U = G == 64;
    using Rec = std::conditional_t<U, UniformAosRec, AosRec>;
    auto record = [&](int p) {
        return Rec{a.rstride ? a.recs + a.rbase + p * a.rstride : a.recs + a.roff[a.cbase + p]};
    };
    auto position = [&](int wt, int f) {
        const int q = (wt * GPW + grp) * PPW + f;
        return U ? __builtin_amdgcn_readfirstlane(q) : q;
    };
    // the first record's loads are issued before anything waits: the run-state loads and the
    // stripe reductions below overlap with them
    int p = position(gw, 0);
    Rec R = record(p < a.csize ? p : 0);
    HeadT<B> hd = load_head<KIND, B>(R);
    // (no branch before the loop: it would split the block and delay the record loads)
    const uint64_t mism = a.stripes[lane].mism;
    const int64_t elite_fitness = a.st->elite_fitness;
    const bool act = (int)i < a.N;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    uint64_t cand = act ? (popm & ~(1ull << i)) : 0ull;
    const bool neutral_ok = (a.always != 0) | (bit_of(wave_or64(mism), i) != 0);
    // a finished run (elitist at the target) and a forced-improvement sweep with nothing
    // left to do skip the loop; both conditions are wave-uniform
    bool live = elite_fitness < a.target;
    if constexpr (FI) {
        // forced improvement: solutions without an accepted step and not yet improved; the
        // elitist is the only donor
        const uint64_t todo = popm & ~wave_or64(a.stripes[lane].acc) &
                              ~fi_done_before(a.fi_at, a.fi_pos);
        live = live && todo != 0;
        cand = act && bit_of(todo, i) ? ~0ull : 0ull;
    }

    int64_t facc = 0;
    uint32_t n_eval = 0, n_acc = 0;  // wave totals (from ballots, wave-uniform)
    bool flag = false;  // GOM: an accepted step; forced improvement: a step that improved
    const PlaneBits bits{a.O, i};
    const PlaneCommit<G> commit{a.O, grp, i};
    const int nwt = (a.csize + GPW * PPW - 1) / (GPW * PPW);  // wave tiles
    U32x4 draw{0u, 0u, 0u, 0u};  // the Philox call of the group's current eight positions
    int f = 0;                   // position within the group's tile (PPW > 1)
    for (int wt = gw; live && wt < nwt;) {
        bool take = p < a.csize;
        if constexpr (PPW > 1) {
            // the tile's call: solution i, counter word 3 = p / 8 (the same for its 8 positions)
            if (f == 0 && take)
                draw = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i, (uint32_t)(p >> 3));
        }
        if constexpr (KIND != 0) {
            const int nm = hd.h0.x;
            if (a.coop && nm >= kCoopMinMembers && nm <= kCoopMaxMembers) take = false;
        }
        PairOut r{0u, false, 0};
        if (take) {
            if constexpr (FI) {
                r = gom_pair<KIND>(R, hd, EliteWords{a.E}, bits, commit, cand, 0u, neutral_ok);
                flag |= r.acc && r.delta > 0;
            } else {
                uint32_t h = 0;
                if constexpr (KIND != 0) {
                    // each lane draws its own call; the 8 positions of a chunk share it
                    const U32x4 q = PPW > 1 ? draw
                                            : philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i,
                                                     (uint32_t)(p >> 3));
                    const int fl = p & 7;
                    const uint32_t w = (fl >> 1) == 0 ? q.x : (fl >> 1) == 1 ? q.y
                                     : (fl >> 1) == 2 ? q.z : q.w;
                    h = (w >> (16 * (fl & 1))) & 0xFFFFu;
                }
                r = gom_pair<KIND>(R, hd, a.P, bits, commit, cand, h, neutral_ok);
                flag |= r.acc;
            }
            facc += r.acc ? r.delta : 0;
        }
        n_eval += (uint32_t)__popcll(ballot64(r.cnt > 0));
        n_acc += (uint32_t)__popcll(ballot64(r.acc));
        if (++f == PPW) {
            f = 0;
            wt += nwaves;
        }
        if (wt < nwt) {
            p = position(wt, f);
            R = record(p < a.csize ? p : 0);
            hd = load_head<KIND, B>(R);
        }
    }

    // per-wave results into stripe (global wave index mod kStripes)
#pragma unroll
    for (int off = 32; off >= G; off >>= 1) facc += __shfl_xor(facc, off, 64);
    const uint32_t ce = n_eval, ca = n_acc;
    Stripe *sp = a.stripes + (gw % kStripes);
    if (lane < G && act && facc)
        atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)facc);
    const uint64_t fm = a.mode == kSweepGomTrack ? solution_mask<G>(flag && act) : 0ull;
    // every group's lanes record their own solutions' improvements (i = lane mod G)
    if (FI && act && flag) atomicMax(&a.fi_at[i], kFiBase - (uint32_t)a.fi_pos);
    if (lane == 0) {
        if (ce) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)ce);
        if (ca) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)ca);
        if (fm) atomicOr((unsigned long long *)&sp->acc, (unsigned long long)fm);
    }
}

// Wave-uniform broadcast of lane l's 32- and 64-bit values (l wave-uniform).
__device__ __forceinline__ int32_t lane_i32(int32_t v, int l) {
    return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int l) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}
// Word idx (< 192) of a record staged as three registers of 64 words (lane l of rK holds word
// 64 K + l), fetched by every lane for its own idx.
__device__ __forceinline__ int32_t staged_word(int32_t r0, int32_t r1, int32_t r2, int idx) {
    const int src = (idx & 63) << 2;  // ds_bpermute addresses bytes
    const int32_t a = __builtin_amdgcn_ds_bpermute(src, r0);
    const int32_t b = __builtin_amdgcn_ds_bpermute(src, r1);
    const int32_t c = __builtin_amdgcn_ds_bpermute(src, r2);
    return idx < 64 ? a : (idx < 128 ? b : c);
}

// GOM step of every solution of the wave (lane i = solution i) on one small set (at most
// kBclMaxMembers members, kBclMaxEntries dependent edges), with the set's data staged by the
// wave in two rounds of loads instead of one round per batch of entries:
//   1. the record's first 192 words, three coalesced loads per lane (the record buffer keeps
//      a zero tail of that length, so a load past the last record stays inside it);
//   2. lane k < nm loads member k's P and O words, lane e < nd (and e + 64) the O word at
//      the far end of dependent edge e when that end lies outside the set;
// then every lane reads members, entries and words with lane reads (wave-uniform values)
// and decides its own step exactly as the other sweeps do: donors D, the draw's r-th donor,
// the changed members C, delta over the dependent edges, acceptance, and a masked store of
// each changed member's word.
__device__ __forceinline__ PairOut staged_pair(const int32_t *rec, const uint64_t *P, uint64_t *O,
                                               uint32_t i, uint64_t cand, uint32_t h,
                                               bool neutral_ok) {
    const int lane = (int)(threadIdx.x & 63);
    const int32_t r0 = rec[lane], r1 = rec[64 + lane], r2 = rec[128 + lane];
    const int nm = __builtin_amdgcn_readfirstlane(r0);        // word 0
    const int nd = __builtin_amdgcn_readlane(r0, 1);           // word 1
    // round 2: member words (lanes < nm) and far-end words (lanes < nd, and lane + 64 < nd)
    const int u = staged_word(r0, r1, r2, 2 + (lane < kBclMaxMembers ? lane : 0));
    const int32_t xlo = staged_word(r0, r1, r2, 16 + 2 * lane);
    const int32_t wlo = staged_word(r0, r1, r2, 17 + 2 * lane);
    const int hl = lane < kBclMaxEntries - 64 ? lane : 0;      // entries 64.. (at most 8)
    const int32_t xhi = staged_word(r0, r1, r2, 16 + 2 * (64 + hl));
    const int32_t whi = staged_word(r0, r1, r2, 17 + 2 * (64 + hl));
    const bool mem = lane < nm;
    const uint64_t pw = mem ? P[u] : 0ull, ow = mem ? O[u] : 0ull;
    const bool olo = lane < nd && xlo >= 0, ohi = 64 + lane < nd && xhi >= 0;
    const uint64_t flo = olo ? O[(uint32_t)xlo & kSmallIdx] : 0ull;
    const uint64_t fhi = ohi ? O[(uint32_t)xhi & kSmallIdx] : 0ull;
    PairOut out{0u, false, 0};
    uint32_t om = 0;
    uint64_t D = 0;
    for (int k = 0; k < nm; ++k) {
        const uint32_t ok = bit_of(lane_u64(ow, k), i);
        om |= ok << k;
        D |= lane_u64(pw, k) ^ (0ull - (uint64_t)ok);
    }
    D &= cand;
    out.cnt = (uint32_t)__popcll(D);
    const uint32_t d = out.cnt ? select_bit(D, (h * out.cnt) >> 16) : 0u;
    uint32_t cm = 0;
    for (int k = 0; k < nm; ++k) cm |= (bit_of(lane_u64(pw, k), d) ^ ((om >> k) & 1u)) << k;
    int64_t delta = 0;
    for (int e = 0; e < nd; ++e) {
        const bool hi = e >= 64;
        const int l = e & 63;
        const int32_t x = lane_i32(hi ? xhi : xlo, l);
        const int32_t w = lane_i32(hi ? whi : wlo, l);
        const uint32_t a = ((uint32_t)x >> kSmallPosShift) & 15u;
        const uint32_t y = (uint32_t)x & kSmallIdx;
        const uint32_t oa = (om >> a) & 1u, ca = (cm >> a) & 1u;
        uint32_t ov, flip;
        if (x < 0) {  // inside edge to member y (wave-uniform branch)
            ov = (om >> y) & 1u;
            flip = ca ^ ((cm >> y) & 1u);
        } else {
            ov = bit_of(lane_u64(hi ? fhi : flo, l), i);
            flip = ca;
        }
        delta += flip ? signed_w(oa == ov, w) : 0;
    }
    out.delta = delta;
    out.acc = out.cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
    // commit: each changed member's new word, stored by the lane that loaded it
    for (int k = 0; k < nm; ++k) {
        const uint64_t fm = ballot64(out.acc && ((cm >> k) & 1u));
        if (fm && lane == k) O[u] = ow ^ fm;
    }
    return out;
}

// One colour class of small general sets with the staged evaluation (staged_pair): lane =
// solution, one set per wave at a time; PPW consecutive positions per wave tile (8: one Philox
// call for all of them, for classes large enough that every wave strides over eight
// positions anyway).  Forced improvement keeps the other sweep.
template <int PPW>
__global__ __launch_bounds__(kSweepMaxThreads) void k_class_sweep_staged(SweepArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t i = (uint32_t)lane;
    const int wpb = (int)(blockDim.x >> 6);
    const int gw = xcd_tile((int)blockIdx.x, (int)gridDim.x) * wpb + (int)(threadIdx.x >> 6);
    const int nwaves = gridDim.x * wpb;
    const uint64_t mism = a.stripes[lane].mism;
    const bool live = a.st->elite_fitness < a.target;
    const bool act = (int)i < a.N;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t cand = act ? (popm & ~(1ull << i)) : 0ull;
    const bool neutral_ok = (a.always != 0) | (bit_of(wave_or64(mism), i) != 0);
    int64_t facc = 0;
    uint32_t n_eval = 0, n_acc = 0;
    bool flag = false;
    const int nwt = (a.csize + PPW - 1) / PPW;
    for (int wt = gw; live && wt < nwt; wt += nwaves) {
        const int p0 = __builtin_amdgcn_readfirstlane(wt * PPW);
        U32x4 q = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i, (uint32_t)(p0 >> 3));
#pragma unroll 1
        for (int f = 0; f < PPW; ++f) {
            const int p = p0 + f;
            if (p >= a.csize) break;
            if (PPW == 1 && f > 0)
                q = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i, (uint32_t)(p >> 3));
            const int32_t *rec = a.rstride ? a.recs + a.rbase + p * a.rstride
                                           : a.recs + a.roff[a.cbase + p];
            const int fl = p & 7;
            const uint32_t w = (fl >> 1) == 0 ? q.x : (fl >> 1) == 1 ? q.y
                             : (fl >> 1) == 2 ? q.z : q.w;
            const uint32_t h = (w >> (16 * (fl & 1))) & 0xFFFFu;
            const PairOut r = staged_pair(rec, a.P, a.O, i, cand, h, neutral_ok);
            facc += r.acc ? r.delta : 0;
            flag |= r.acc;
            n_eval += (uint32_t)__popcll(ballot64(r.cnt > 0));
            n_acc += (uint32_t)__popcll(ballot64(r.acc));
        }
    }
    Stripe *sp = a.stripes + (gw % kStripes);
    if (act && facc) atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)facc);
    const uint64_t fm = a.mode == kSweepGomTrack ? ballot64(flag && act) : 0ull;
    if (lane == 0) {
        if (n_eval) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)n_eval);
        if (n_acc) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)n_acc);
        if (fm) atomicOr((unsigned long long *)&sp->acc, (unsigned long long)fm);
    }
}

// ------------------------------------------------------------------------------------------
// Block-cooperative sweep of one large set (general record layout) for every solution at
// once: block = set, lane = solution, the block's waves split the set's members.
//   1. D_i = OR over members u of (P[u] xor broadcast(O_i[u])), reduced over the waves; the
//      first wave picks each solution's donor from its 16-bit Philox field (the set's class
//      position p, as in the other sweeps)
//   2. per member k: the mask of solutions whose donor changes u_k, kept in LDS (cmw[k])
//   3. delta_i over the set's dependent edges (each member's entries, members split over
//      the waves; an inside edge changes when exactly one end changes), reduced over waves
//   4. accept as in the other sweeps; each wave commits its members: O[u] ^= cmw & accepted
// Forced improvement (mode kSweepFi): the elitist is the donor.  Sets of one class are
// independent, so blocks never touch each other's words.
// ------------------------------------------------------------------------------------------
constexpr int kCoopMaxThreads = 1024;
constexpr int kCoopUnroll = 4;   // members per wave and step
constexpr int kCoopEdges = 8;    // entries of a member fetched together

__global__ __launch_bounds__(kCoopMaxThreads) void k_large_set_sweep(SweepArgs a) {
    extern __shared__ uint64_t cmw[];        // change masks, then offspring words (om)
    uint64_t *om = cmw + a.coop_cap;
    const int W = (int)(blockDim.x >> 6);
    __shared__ uint64_t red[kCoopMaxThreads / 64][64];
    __shared__ int64_t redd[kCoopMaxThreads / 64][64];
    __shared__ uint32_t sel[64];
    __shared__ uint64_t accm_s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i = (uint32_t)lane;
    const int p = a.large_pos[blockIdx.x];
    const int32_t *R = a.rstride ? a.recs + a.rbase + p * a.rstride : a.recs + a.roff[a.cbase + p];
    const uint64_t mism = a.stripes[lane].mism;
    const uint64_t acc_prev = a.mode == kSweepFi ? a.stripes[lane].acc : 0ull;
    if (a.st->elite_fitness >= a.target) return;
    const int nm = R[0];
    const int32_t *mem = R + 16;
    const int32_t *end = R + 16 + nm;
    const int2 *E = reinterpret_cast<const int2 *>(R + ((16 + 2 * nm + 3) & ~3));
    const bool act = (int)i < a.N;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    uint64_t cand = act ? (popm & ~(1ull << i)) : 0ull;
    const bool neutral_ok = a.always || bit_of(wave_or64(mism), i);
    const bool fi = a.mode == kSweepFi;
    if (fi) {
        const uint64_t todo = popm & ~wave_or64(acc_prev) & ~fi_done_before(a.fi_at, a.fi_pos);
        if (todo == 0) return;  // uniform over the block
        cand = act && bit_of(todo, i) ? ~0ull : 0ull;
    }
    const EliteWords ew{a.E};
    auto donor_word = [&](int u) { return fi ? ew[u] : a.P[u]; };

    // Members are taken kCoopUnroll at a time by each wave (chunks k0 .. k0 + 3), so that
    // the loads of several members are in flight together.
    // 1. eligible donors
    uint64_t D = 0;
    for (int k0 = w * kCoopUnroll; k0 < nm; k0 += W * kCoopUnroll) {
#pragma unroll
        for (int c = 0; c < kCoopUnroll; ++c) {
            const int k = k0 + c;
            const int u = mem[k < nm ? k : 0];
            const uint64_t o = a.O[u];
            const uint64_t t = donor_word(u) ^ (0ull - (uint64_t)bit_of(o, i));
            if (k < nm) {
                D |= t;
                if (lane == 0) om[k] = o;
            }
        }
    }
    red[w][lane] = D;
    __syncthreads();
    uint32_t cnt = 0, d = 0;
    if (w == 0) {
        D = 0;
        for (int q = 0; q < W; ++q) D |= red[q][lane];
        D &= cand;
        cnt = (uint32_t)__popcll(D);
        uint32_t h = 0;
        if (!fi) {
            const U32x4 r = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i,
                                   (uint32_t)(p >> 3));
            const int f = p & 7;
            const uint32_t x = (f >> 1) == 0 ? r.x : (f >> 1) == 1 ? r.y : (f >> 1) == 2 ? r.z : r.w;
            h = (x >> (16 * (f & 1))) & 0xFFFFu;
        }
        d = cnt ? select_bit(D, (h * cnt) >> 16) : 0u;
        sel[lane] = d;
        red[0][lane] = cnt;  // reused: donor counts
    }
    __syncthreads();
    d = sel[lane];
    cnt = (uint32_t)red[0][lane];
    // 2. change masks per member
    for (int k0 = w * kCoopUnroll; k0 < nm; k0 += W * kCoopUnroll) {
#pragma unroll
        for (int c = 0; c < kCoopUnroll; ++c) {
            const int k = k0 + c;
            const int kk = k < nm ? k : 0;
            const uint32_t flip = bit_of(donor_word(mem[kk]), d) ^ bit_of(om[kk], i);
            const uint64_t m = ballot64(flip != 0 && cnt > 0);
            if (lane == 0 && k < nm) cmw[k] = m;
        }
    }
    __syncthreads();
    // 3. fitness change over the dependent edges: each member's first kCoopEdges entries
    // are fetched together (masked past the member's end), longer lists continue in a loop
    int64_t dl = 0;
    auto edge = [&](int2 en, uint32_t oa, uint32_t ca) -> int64_t {
        uint32_t ov, flip;
        if (en.x >= 0) {
            ov = bit_of(a.O[en.x], i);
            flip = ca;
        } else {
            const int b = ~en.x;
            ov = bit_of(om[b], i);
            flip = ca ^ bit_of(cmw[b], i);
        }
        return flip ? signed_w(oa == ov, en.y) : 0;
    };
    for (int k0 = w * kCoopUnroll; k0 < nm; k0 += W * kCoopUnroll) {
#pragma unroll
        for (int c = 0; c < kCoopUnroll; ++c) {
            const int k = k0 + c;
            if (k >= nm) break;
            const uint32_t oa = bit_of(om[k], i), ca = bit_of(cmw[k], i);
            const int e0 = k ? end[k - 1] : 0, e1 = end[k];
#pragma unroll
            for (int t = 0; t < kCoopEdges; ++t) {
                const int e = e0 + t;
                const int2 en = E[e < e1 ? e : e0];
                if (e < e1) dl += edge(en, oa, ca);
            }
            for (int e = e0 + kCoopEdges; e < e1; ++e) dl += edge(E[e], oa, ca);
        }
    }
    redd[w][lane] = dl;
    __syncthreads();
    if (w == 0) {
        int64_t delta = 0;
        for (int q = 0; q < W; ++q) delta += redd[q][lane];
        const bool acc = cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
        const uint64_t am = ballot64(acc);
        if (lane == 0) accm_s = am;
        Stripe *sp = a.stripes + (blockIdx.x % kStripes);
        if (acc && delta) atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)delta);
        const uint64_t ev = ballot64(cnt > 0);
        if (fi && acc && delta > 0) atomicMax(&a.fi_at[i], kFiBase - (uint32_t)a.fi_pos);
        if (lane == 0) {
            if (ev) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)__popcll(ev));
            if (am) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)__popcll(am));
            if (a.mode == kSweepGomTrack && am)
                atomicOr((unsigned long long *)&sp->acc, (unsigned long long)am);
        }
    }
    __syncthreads();
    // 4. commit
    const uint64_t am = accm_s;
    if (am)
        for (int k = threadIdx.x; k < nm; k += (int)blockDim.x) {
            const uint64_t m = cmw[k] & am;
            if (m) a.O[mem[k]] ^= m;
        }
}

// ------------------------------------------------------------------------------------------
// Split sweep of a few large sets (general record layout): the members of each set are cut
// into chunks of kSplitMembers, one 256-thread block per chunk (lane = solution, each wave
// kSplitPerWave members), so that a class holding a handful of sets of thousands of members
// still spreads over the device.  Three launches, the steps of the block-cooperative sweep
// with the set-wide reductions in global memory (per slot = the set's index in its group):
//   1. k_split_donors: D_i = OR over the chunk's members of (P[u] xor broadcast(O_i[u])),
//      OR-ed into split_D; the first chunk's block clears the set's split_delta
//   2. k_split_delta: every block draws the donors from split_D (16-bit Philox field of the
//      set's class position, as in the other sweeps) and sums the change of its members'
//      dependent edges into split_delta (an inside edge changes when exactly one end changes;
//      the other end's change is recomputed from its words); the first chunk's block stores
//      the donor choices in split_sel
//   3. k_split_commit: acceptance per solution from split_sel and split_delta, each block
//      commits its members (O[u] ^= changed & accepted); the first chunk's block adds the
//      set's fitness changes and counts to a stripe and clears the set's split_D
// OR and integer sums do not depend on the order of the atomic updates, so the result equals
// the one-block sweep.  Forced improvement (mode kSweepFi): the elitist is the donor.
// ------------------------------------------------------------------------------------------
constexpr int kSplitThreads = 256;
constexpr int kSplitWaves = kSplitThreads / 64;
constexpr int kSplitPerWave = kSplitMembers / kSplitWaves;
static_assert(kSplitPerWave * kSplitWaves == kSplitMembers, "members per block");

struct SplitBlock {
    int slot, p, k0, nm;
    const int32_t *mem, *end;
    const int2 *E;
};

__device__ __forceinline__ SplitBlock split_block(const SweepArgs &a) {
    const int4 m = a.smap[blockIdx.x];
    const int32_t *R = a.rstride ? a.recs + a.rbase + m.y * a.rstride
                                 : a.recs + a.roff[a.cbase + m.y];
    const int nm = R[0];
    return SplitBlock{m.x, m.y, m.z, nm, R + 16, R + 16 + nm,
                      reinterpret_cast<const int2 *>(R + ((16 + 2 * nm + 3) & ~3))};
}

__global__ __launch_bounds__(kSplitThreads) void k_split_donors(SweepArgs a) {
    __shared__ uint64_t red[kSplitWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i = (uint32_t)lane;
    const SplitBlock sb = split_block(a);
    if (a.st->elite_fitness >= a.target) return;  // uniform over the grid
    const bool fi = a.mode == kSweepFi;
    const EliteWords ew{a.E};
    uint64_t D = 0;
#pragma unroll
    for (int c = 0; c < kSplitPerWave; ++c) {
        const int k = sb.k0 + w * kSplitPerWave + c;
        const int u = sb.mem[k < sb.nm ? k : 0];
        const uint64_t o = a.O[u];
        const uint64_t t = (fi ? ew[u] : a.P[u]) ^ (0ull - (uint64_t)bit_of(o, i));
        if (k < sb.nm) D |= t;
    }
    red[w][lane] = D;
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int q = 1; q < kSplitWaves; ++q) D |= red[q][lane];
        if (D) atomicOr((unsigned long long *)&a.split_D[sb.slot * 64 + lane],
                        (unsigned long long)D);
        if (sb.k0 == 0) a.split_delta[sb.slot * 64 + lane] = 0;
    }
}

__global__ __launch_bounds__(kSplitThreads) void k_split_delta(SweepArgs a) {
    __shared__ int64_t red[kSplitWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i = (uint32_t)lane;
    const SplitBlock sb = split_block(a);
    const uint64_t Dall = a.split_D[sb.slot * 64 + lane];
    const uint64_t acc_prev = a.stripes[lane].acc;
    if (a.st->elite_fitness >= a.target) return;
    const bool fi = a.mode == kSweepFi;
    const bool act = (int)i < a.N;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    uint64_t cand = act ? (popm & ~(1ull << i)) : 0ull;
    if (fi) {
        const uint64_t todo = popm & ~wave_or64(acc_prev) & ~fi_done_before(a.fi_at, a.fi_pos);
        cand = act && bit_of(todo, i) ? ~0ull : 0ull;
    }
    const uint64_t D = Dall & cand;
    const uint32_t cnt = (uint32_t)__popcll(D);
    uint32_t h = 0;
    if (!fi) {
        const U32x4 r = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls, i, (uint32_t)(sb.p >> 3));
        const int f = sb.p & 7;
        const uint32_t x = (f >> 1) == 0 ? r.x : (f >> 1) == 1 ? r.y : (f >> 1) == 2 ? r.z : r.w;
        h = (x >> (16 * (f & 1))) & 0xFFFFu;
    }
    const uint32_t d = cnt ? select_bit(D, (h * cnt) >> 16) : 0u;
    if (sb.k0 == 0 && w == 0)
        a.split_sel[sb.slot * 64 + lane] = (int32_t)(d | (cnt ? 0x10000u : 0u));
    const EliteWords ew{a.E};
    // does the step of solution i change vertex u (O_i[u] in o)?
    auto changes = [&](int u, uint64_t o) -> uint32_t {
        return cnt ? bit_of(fi ? ew[u] : a.P[u], d) ^ bit_of(o, i) : 0u;
    };
    auto edge = [&](int2 en, uint32_t oa, uint32_t ca) -> int64_t {
        uint32_t ov, flip;
        if (en.x >= 0) {
            ov = bit_of(a.O[en.x], i);
            flip = ca;
        } else {
            const int ub = sb.mem[~en.x];
            const uint64_t ob = a.O[ub];
            ov = bit_of(ob, i);
            flip = ca ^ changes(ub, ob);
        }
        return flip ? signed_w(oa == ov, en.y) : 0;
    };
    int64_t dl = 0;
#pragma unroll
    for (int c = 0; c < kSplitPerWave; ++c) {
        const int k = sb.k0 + w * kSplitPerWave + c;
        if (k >= sb.nm) break;  // uniform over the wave
        const int u = sb.mem[k];
        const uint64_t o = a.O[u];
        const uint32_t oa = bit_of(o, i), ca = changes(u, o);
        const int e0 = k ? sb.end[k - 1] : 0, e1 = sb.end[k];
        // the member's first kCoopEdges entries together (masked past its end)
#pragma unroll
        for (int t = 0; t < kCoopEdges; ++t) {
            const int e = e0 + t;
            const int2 en = sb.E[e < e1 ? e : e0];
            if (e < e1) dl += edge(en, oa, ca);
        }
        for (int e = e0 + kCoopEdges; e < e1; ++e) dl += edge(sb.E[e], oa, ca);
    }
    red[w][lane] = dl;
    __syncthreads();
    if (w == 0) {
        int64_t s = 0;
#pragma unroll
        for (int q = 0; q < kSplitWaves; ++q) s += red[q][lane];
        if (s) atomicAdd((unsigned long long *)&a.split_delta[sb.slot * 64 + lane],
                         (unsigned long long)s);
    }
}

__global__ __launch_bounds__(kSplitThreads) void k_split_commit(SweepArgs a) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i = (uint32_t)lane;
    const SplitBlock sb = split_block(a);
    const uint64_t mism = a.stripes[lane].mism;
    const int32_t sel = a.split_sel[sb.slot * 64 + lane];
    const int64_t delta = a.split_delta[sb.slot * 64 + lane];
    if (a.st->elite_fitness >= a.target) return;
    const bool fi = a.mode == kSweepFi;
    const bool neutral_ok = a.always || bit_of(wave_or64(mism), i);
    const uint32_t d = (uint32_t)sel & 0xFFFFu;
    const bool has = ((uint32_t)sel >> 16) != 0u;
    const bool acc = has && (delta > 0 || (delta == 0 && neutral_ok));
    const uint64_t am = ballot64(acc);
    const EliteWords ew{a.E};
#pragma unroll
    for (int c = 0; c < kSplitPerWave; ++c) {
        const int k = sb.k0 + w * kSplitPerWave + c;
        if (k >= sb.nm) break;  // uniform over the wave
        const int u = sb.mem[k];
        const uint64_t o = a.O[u];
        const bool flip = has && (bit_of(fi ? ew[u] : a.P[u], d) ^ bit_of(o, i)) != 0u;
        const uint64_t m = ballot64(flip) & am;
        if (lane == 0 && m) a.O[u] = o ^ m;  // only this block touches u
    }
    if (sb.k0 == 0 && w == 0) {
        Stripe *sp = a.stripes + (sb.slot % kStripes);
        if (acc && delta) atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)delta);
        const uint64_t ev = ballot64(has);
        if (fi && acc && delta > 0) atomicMax(&a.fi_at[i], kFiBase - (uint32_t)a.fi_pos);
        if (lane == 0) {
            if (ev) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)__popcll(ev));
            if (am) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)__popcll(am));
            if (a.mode == kSweepGomTrack && am)
                atomicOr((unsigned long long *)&sp->acc, (unsigned long long)am);
        }
        a.split_D[sb.slot * 64 + lane] = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Colouring-parallel local search, one colour class of a univariate FOS (the hybrid that the
// paper's conclusion names as future work).  Wave = set {u} (class positions strided over the
// grid's waves, XCD-contiguous), lane = solution i:
//   gain_i = sum over u's edges (u, v, w) of (+w if O_i[u] == O_i[v], else -w)
//   every solution with gain_i > 0 flips u: one word store O[u] ^= ballot(gain > 0)
// Sets of one class share no variable and no edge, so no wave reads a word that another
// writes.  The gains of the flips go to the wave's stripe; any flip sets ls_any.
// ------------------------------------------------------------------------------------------
constexpr int kLsThreads = 256;

__global__ __launch_bounds__(kLsThreads) void k_ls_sweep(SweepArgs a) {
    constexpr int wpb = kLsThreads / 64;
    const int lane = threadIdx.x & 63;
    const uint32_t i = (uint32_t)lane;
    const int gw = xcd_tile((int)blockIdx.x, (int)gridDim.x) * wpb + (int)(threadIdx.x >> 6);
    const int nwaves = (int)gridDim.x * wpb;
    const bool act = (int)i < a.N;
    int64_t facc = 0;
    bool any = false;
    for (int p = gw; p < a.csize; p += nwaves) {  // uniform over the wave
        const int32_t *R = a.rstride ? a.recs + a.rbase + p * a.rstride
                                     : a.recs + a.roff[a.cbase + p];
        const int u = __builtin_amdgcn_readfirstlane(R[0]);
        const int nd = __builtin_amdgcn_readfirstlane(R[1]);
        const int2 *en = reinterpret_cast<const int2 *>(R + 4);
        const uint64_t ow = a.O[u];
        const uint32_t ou = bit_of(ow, i);
        int64_t gain = 0;
        for (int e0 = 0; e0 < nd; e0 += kBatch) {
            int2 x[kBatch];
            uint32_t ov[kBatch];
#pragma unroll
            for (int t = 0; t < kBatch; ++t)
                if (e0 + t < nd) x[t] = en[e0 + t];
#pragma unroll
            for (int t = 0; t < kBatch; ++t)
                if (e0 + t < nd) ov[t] = bit_of(a.O[x[t].x], i);
#pragma unroll
            for (int t = 0; t < kBatch; ++t)
                if (e0 + t < nd) gain += signed_w(ou == ov[t], x[t].y);
        }
        const bool flip = act && gain > 0;
        const uint64_t m = ballot64(flip);
        if (lane == 0 && m) a.O[u] = ow ^ m;
        facc += flip ? gain : 0;
        any |= m != 0;
    }
    Stripe *sp = a.stripes + (gw % kStripes);
    if (act && facc) atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)facc);
    if (any && lane == 0) atomicOr(a.ls_any, 1u);
}

// ------------------------------------------------------------------------------------------
// Perturbation of one round of the iterated local search, one wave, lane = solution i.  Flip
// t < flips: word t mod 4 of Philox(seed; g, kPerturbStream, i, 16 r + t / 4), scaled to a
// class position q = (word * |F|) >> 32, names a set; its variable u flips in O_i and the
// flip's gain (against the genes after the earlier flips) adds to the solution's fitness
// change.  Genes are read from P, which the round leaves alone (O equals P when it starts),
// with the lane's earlier flips (its own column of an LDS list) applied on top, so no lane
// reads a word that is being written.  The flips go into O by atomic XOR: two lanes may flip
// the same word.
// ------------------------------------------------------------------------------------------
constexpr int kPerturbMaxFlips = 64;

__global__ __launch_bounds__(64) void k_perturb(PerturbArgs a) {
    __shared__ int32_t done[kPerturbMaxFlips][64];
    const int lane = threadIdx.x;
    if (lane >= a.N) return;
    const uint32_t i = (uint32_t)lane;
    auto gene = [&](int v, int flipped) {
        uint32_t b = bit_of(a.P[v], i);
        for (int s = 0; s < flipped; ++s) b ^= (uint32_t)(done[s][lane] == v);
        return b;
    };
    int64_t d = 0;
    U32x4 r{};
    for (int t = 0; t < a.flips; ++t) {
        if ((t & 3) == 0)
            r = philox(a.seed, (uint32_t)a.gen, kPerturbStream, i,
                       (uint32_t)a.round * 16u + (uint32_t)(t >> 2));
        const uint32_t w = (t & 3) == 0 ? r.x : (t & 3) == 1 ? r.y : (t & 3) == 2 ? r.z : r.w;
        const int q = (int)(((uint64_t)w * (uint64_t)a.n_sets) >> 32);
        const int32_t *R = a.recs + a.roff[q];
        const int u = R[0], nd = R[1];
        const int2 *en = reinterpret_cast<const int2 *>(R + 4);
        const uint32_t ou = gene(u, t);
        int64_t gain = 0;
        for (int e = 0; e < nd; ++e) {
            const int2 x = en[e];
            gain += signed_w(ou == gene(x.x, t), x.y);
        }
        d += gain;
        done[t][lane] = u;
        atomicXor((unsigned long long *)&a.O[u], 1ull << i);
    }
    if (d) atomicAdd((unsigned long long *)&a.stripes[0].fit[i], (unsigned long long)d);
}

// ------------------------------------------------------------------------------------------
// Bit-parallel sweep of one colour class for a univariate FOS on a graph of degree <= 4
// (lane = set, all solutions of a set in one 64-bit word).
//
// For set {u} with edges (u, v_e, w_e), e < 4 (missing edges have w = 0):
//   q_e    = ~(O[u] ^ O[v_e]): bit i set when u and v_e carry the same gene in O_i, so
//            flipping u cuts the edge (+w_e); otherwise it uncuts it (-w_e)
//   delta  of solution i depends only on the 4-bit pattern (q_0..q_3 at bit i): the set's
//            table entry carries two 16-entry truth tables over the patterns (delta > 0,
//            delta == 0), computed from the set's weights on the host; the lane evaluates
//            them on all 64 solutions at once with a tree of bitwise selects on q_0..q_3
//   donor  exists for solution i when some other solution's P gene at u differs from
//            O_i[u]: from the popcounts of the ones and zeros of P[u]
//   accept = donor & (positive | (zero & not-elitist)), O[u] ^= accept
// The donor draw is not needed: with one variable every eligible donor carries the flipped
// gene.  Fitness changes of accepted pairs (delta of that pair recomputed from its pattern)
// are summed per solution in LDS and added to the block's stripe.
// PARTITION: every variable is in exactly one set, so O[u] still equals P[u] when u's set
// is swept and P[u] need not be read.
// The sets come from the bit-sliced table (one array per field, entry = class position), so a
// lane reads 24 bytes (u, tables, four neighbours) with six coalesced loads; the weights are
// read only when one of the lane's solutions accepts.
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ uint64_t sel64(uint64_t m, uint64_t a, uint64_t b) {
    return (a & m) | (b & ~m);  // per bit: m ? a : b
}

// All ones when bit b of t is set, else zero (one signed bit-field extract).
__device__ __forceinline__ uint32_t bit_mask32(uint32_t t, int b) {
    return (uint32_t)(((int32_t)(t << (31 - b))) >> 31);
}

// 16-entry truth table t (bit p = value for pattern p = q0 + 2 q1 + 4 q2 + 8 q3) evaluated
// bitwise on the four masks.  Leaf k covers patterns 2k (q0 = 0) and 2k + 1 (q0 = 1): with
// their table bits spread to all-ones/zero words A and B it is (q0 & B) | (~q0 & A), one
// bit-field insert per 32-bit half; then a select tree on q1, q2, q3.
__device__ __forceinline__ uint64_t table16(uint32_t t, uint64_t q0, uint64_t q1, uint64_t q2,
                                            uint64_t q3) {
    const uint32_t q0l = (uint32_t)q0, q0h = (uint32_t)(q0 >> 32);
    uint64_t l[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t A = bit_mask32(t, 2 * k), B = bit_mask32(t, 2 * k + 1);
        l[k] = (uint64_t)((q0l & B) | (~q0l & A)) | ((uint64_t)((q0h & B) | (~q0h & A)) << 32);
    }
    uint64_t m1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m1[k] = sel64(q1, l[2 * k + 1], l[2 * k]);
    const uint64_t m20 = sel64(q2, m1[1], m1[0]), m21 = sel64(q2, m1[3], m1[2]);
    return sel64(q3, m21, m20);
}

// One entry of the bit-sliced table: the set's variable, its neighbours, its truth tables.
struct SwarEntry {
    int u, v0, v1, v2, v3;
    uint32_t tab;
};

// Entry q of the table (q: the set's position in the class order of all classes).
__device__ __forceinline__ SwarEntry swar_entry(const SweepArgs &a, int q) {
    const size_t ss = (size_t)a.sw_stride;
    const int32_t *T = a.sw + q;
    return SwarEntry{T[kSwU * ss], T[kSwV * ss], T[(kSwV + 1) * ss], T[(kSwV + 2) * ss],
                     T[(kSwV + 3) * ss], (uint32_t)T[kSwTables * ss]};
}

// The GOM step of every solution at once on the set of table entry q (univariate FOS): the
// accepted mask is flipped into O[u] and each accepted solution's fitness change is added to
// its LDS counter fa[j]; n_eval / n_acc count the lane's pairs with a donor / accepted.
template <bool PARTITION, class Acc>
__device__ __forceinline__ void swar_step(const SweepArgs &a, const SwarEntry &en, int q,
                                          uint64_t popm, uint64_t nz, Acc *fa,
                                          uint32_t &n_eval, uint32_t &n_acc) {
    const size_t ss = (size_t)a.sw_stride;
    // change of solution base + j for every set bit j of m (one 32-bit half of the accepted
    // mask): 2 * (sum of w_k over the edges that become cut) - (sum of all four w_k)
    auto add_flips = [&](uint32_t m, int base, uint32_t h0, uint32_t h1, uint32_t h2,
                         uint32_t h3, int w0, int w1, int w2, int w3, int wsum) {
        for (; m; m &= m - 1) {
            const uint32_t j = (uint32_t)__builtin_ctz(m);
            // bit j of h spread to all ones or zero (signed bit-field extract)
            auto spread = [&](uint32_t h) { return __builtin_amdgcn_sbfe((int)h, j, 1u); };
            const int cut = (w0 & spread(h0)) + (w1 & spread(h1)) + (w2 & spread(h2)) +
                            (w3 & spread(h3));
            atomicAdd(&fa[base + (int)j], (Acc)(2 * cut - wsum));
        }
    };
    const int32_t *T = a.sw + q;
    const int u = en.u, v0 = en.v0, v1 = en.v1, v2 = en.v2, v3 = en.v3;
    const uint32_t tab = en.tab;
    const uint64_t o = a.O[u];
    const uint64_t x = PARTITION ? o : a.P[u];
    const uint64_t q0 = ~(o ^ a.O[v0]), q1 = ~(o ^ a.O[v1]);
    const uint64_t q2 = ~(o ^ a.O[v2]), q3 = ~(o ^ a.O[v3]);
    // donors: solutions with o_i = 1 need a zero of x other than i, o_i = 0 a one
    const uint64_t ones = x & popm, zeros = ~x & popm;
    const int co = __popcll(ones), cz = __popcll(zeros);
    const uint64_t hz = cz >= 2 ? ~0ull : (cz == 1 ? ~zeros : 0ull);
    const uint64_t ho = co >= 2 ? ~0ull : (co == 1 ? ~ones : 0ull);
    const uint64_t has = ((o & hz) | (~o & ho)) & popm;
    // truth tables over the 16 patterns, precomputed on the host
    const uint32_t tp = tab & 0xFFFFu, tz = tab >> 16;
    const uint64_t acc =
        (table16(tp, q0, q1, q2, q3) | (table16(tz, q0, q1, q2, q3) & nz)) & has;
    n_eval += (uint32_t)__popcll(has);
    n_acc += (uint32_t)__popcll(acc);
    if (acc) {
        a.O[u] = o ^ acc;
        // the weights are needed only here: loading them with the entry for every set
        // costs more than this extra round trip for the sets that accept
        const int w0 = T[kSwW * ss], w1 = T[(kSwW + 1) * ss];
        const int w2 = T[(kSwW + 2) * ss], w3 = T[(kSwW + 3) * ss];
        const int wsum = w0 + w1 + w2 + w3;
        add_flips((uint32_t)acc, 0, (uint32_t)q0, (uint32_t)q1, (uint32_t)q2,
                  (uint32_t)q3, w0, w1, w2, w3, wsum);
        add_flips((uint32_t)(acc >> 32), 32, (uint32_t)(q0 >> 32), (uint32_t)(q1 >> 32),
                  (uint32_t)(q2 >> 32), (uint32_t)(q3 >> 32), w0, w1, w2, w3, wsum);
    }
}

// Block totals of a bit-sliced sweep into the block's stripe: the LDS fitness counters of
// the population's solutions and the wave sums of the pair counts.
template <class Acc>
__device__ __forceinline__ void swar_block_totals(const SweepArgs &a, const Acc *fa,
                                                  uint32_t (*redc)[kSwarThreads / 64],
                                                  uint32_t n_eval, uint32_t n_acc) {
    const uint32_t ce = wave_sum32(n_eval), ca = wave_sum32(n_acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        redc[0][wave] = ce;
        redc[1][wave] = ca;
    }
    __syncthreads();
    Stripe *sp = a.stripes + (blockIdx.x % kStripes);
    if ((int)threadIdx.x < a.N && fa[threadIdx.x])
        atomicAdd((unsigned long long *)&sp->fit[threadIdx.x],
                  (unsigned long long)(long long)fa[threadIdx.x]);
    if (threadIdx.x == 0) {
        uint32_t se = 0, sa = 0;
        for (int w = 0; w < kSwarThreads / 64; ++w) {
            se += redc[0][w];
            sa += redc[1][w];
        }
        if (se) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)se);
        if (sa) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)sa);
    }
}

// NARROW: the block's per-solution fitness sums fit in int32 (the host checks the weights'
// bound), so they are kept as 32-bit LDS counters; else 64-bit.
template <bool PARTITION, bool NARROW>
__global__ __launch_bounds__(kSwarThreads) void k_uni_swar_sweep(SweepArgs a) {
    using Acc = std::conditional_t<NARROW, int, unsigned long long>;
    const int stride = gridDim.x * kSwarThreads;
    const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    // the first set's table entry is loaded before anything waits (the run-state loads and
    // the block barrier below overlap with it); positions past the class read a valid entry
    // of the table and are not used
    int p = tile * kSwarThreads + threadIdx.x;
    SwarEntry en = swar_entry(a, a.cbase + (p < a.csize ? p : 0));
    const uint64_t mism = a.stripes[threadIdx.x & 63].mism;
    const bool live = a.st->elite_fitness < a.target;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t nz = a.always ? popm : (wave_or64(mism) & popm);
    __shared__ Acc fa[64];
    __shared__ uint32_t redc[2][kSwarThreads / 64];
    if (threadIdx.x < 64) fa[threadIdx.x] = 0;
    __syncthreads();
    if (!live) return;  // uniform over the grid
    uint32_t n_eval = 0, n_acc = 0;
    for (; p < a.csize; p += stride) {
        if (p != tile * kSwarThreads + (int)threadIdx.x) en = swar_entry(a, a.cbase + p);
        swar_step<PARTITION>(a, en, a.cbase + p, popm, nz, fa, n_eval, n_acc);
    }
    swar_block_totals(a, fa, redc, n_eval, n_acc);
}

// ------------------------------------------------------------------------------------------
// Bit-sliced sweep of one colour class of small general sets (lane = one half of a set's
// solutions as the bits of a 32-bit word: two lanes a set when the population is above 32,
// else one).  Each pair gets the step of the class sweep (k_class_sweep): the donor set D,
// the draw's donor, the changed members C, the partial evaluation and the acceptance rule,
// with the same Philox draws.  Per lane:
//   1. draws: the eight lanes of class positions 8j..8j+7 (one half) share one Philox call per
//      solution (counter (g, c, i, j)); lane l computes the calls of solutions l, l+8, l+16,
//      l+24 of the half and leaves their words in LDS, where each lane reads its own field;
//   2. per solution i (a loop): D_i = OR over the members of (P[u] xor O_i[u] spread), the
//      donor d = the r-th set bit of D_i, and bit i of each member's change mask F_k (the
//      donor's gene differs from O_i's);
//   3. the fitness change of all 32 solutions at once: for dependent edge e with weight w_e,
//      X_e (the edge's cut changes: one end changes) and A_e (it changes towards +|w_e|:
//      becomes cut for w_e > 0, uncut for w_e < 0) give Y_e = 2 A_e + (1 - X_e) in {0, 1, 2},
//      and T = sum_e |w_e| Y_e = delta + W with W = sum_e |w_e|.  T is summed bit-sliced in
//      carry-save form over kGsPlanes bit planes (the host bounds W so that 2 W < 2^kGsPlanes);
//   4. accept = donor exists & (T > W | (T == W & (always | P_i != elitist))); member words
//      are stored with F_k & accept flipped, and each accepted solution's T - W is added to
//      its LDS counter.
// M: member slots (a class's largest set); WB: bits of the class's largest |w|.  Sets of a
// class are independent, so each lane alone reads and writes its members' words, and the
// outside ends of its edges belong to no set of the class.
// ------------------------------------------------------------------------------------------
constexpr int kGsPlanes = 15;

__device__ __forceinline__ uint32_t maj3(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0xE8);  // at least two of the three bits
}
__device__ __forceinline__ uint32_t xor3(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96);
}

template <int M, int WB>
struct GsLds {
    uint4 rnd[kGsThreads / 8][32];     // Philox words: lane group of eight, solution of the half
    uint32_t fo[2][M][kGsThreads];     // F_k and O half-words by member slot, one column a lane
};

// Work item of lane slot q (a multiple-of-16 offset into a class's slots): 16 consecutive
// slots hold 8 positions x 2 halves (population above 32: slots 0-7 half 0, 8-15 half 1) or
// 16 positions (one half).  Every aligned group of 8 slots then shares (position / 8, half),
// i.e. one Philox call per solution, and slot & 7 is the position's field of that call.
struct GsItem {
    int p, h;
};
__device__ __forceinline__ GsItem gs_item(int q, int halves) {
    const int g16 = q >> 4, r = q & 15;
    return halves == 2 ? GsItem{g16 * 8 + (r & 7), r >> 3} : GsItem{g16 * 16 + r, 0};
}

// Draws of the lane's group: lane j of the group (j = slot & 7) computes the calls of
// solutions 32h + i0 + j + 8t, t < 4 / PARTS (i0 = 16 x the lane's part when a half is split
// between two lanes), with counter (g, c, i, p / 8), the group's common values.
template <int PARTS = 1>
__device__ __forceinline__ void gs_draws(uint4 (*rnd)[32], int tid, uint64_t seed, int gen,
                                         int cls, int p, int h, int i0 = 0) {
    const int j = tid & 7;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 4 / PARTS; ++t) {
        const int ii = i0 + j + 8 * t;
        const U32x4 q = philox(seed, (uint32_t)gen, (uint32_t)cls, (uint32_t)(32 * h + ii),
                               (uint32_t)(p >> 3));
        rnd[tid >> 3][ii] = make_uint4(q.x, q.y, q.z, q.w);
    }
    __builtin_amdgcn_wave_barrier();
}

// Work item of a batched class-launch slot, where each half of a set is split between
// kGsPartsBcl lanes (parts): 8 positions take 8 x parts x halves consecutive slots, in groups
// of 8 lanes of one (half, part); the partners of a lane are the lanes 8, 16, ... away.
struct GsItem2 {
    int p, h, pt;
};
__device__ __forceinline__ GsItem2 gs_item2(int q, int halves) {
    const int lp = kGsPartsBcl * halves;    // lanes per position
    const int g = q / (8 * lp), r = q % (8 * lp);
    const int sub = r >> 3;
    return GsItem2{g * 8 + (r & 7), sub / kGsPartsBcl, sub % kGsPartsBcl};
}

// The step of one lane: half h of the set whose record is R (act: the lane has a set; n_i:
// solutions of the half, 32h .. 32h + n_i - 1).  Member words are stored with the accepted
// changes; fit_add(ii, delta) receives each accepted solution's fitness change.
// PARTS > 1: the half is split between PARTS lanes 8 apart (this lane is part pt): each draws
// the donors of 32 / PARTS of the 32 solutions and sums a share of the edges; they exchange
// their change masks and their partial sums, then each commits every PARTS-th member and
// accounts for its own solutions.
template <int M, int WB, int EB, int PARTS = 1, class FitAdd>
__device__ __forceinline__ void gs_step(GsLds<M, WB> &L, int tid, const uint64_t *P, uint64_t *O,
                                        const int32_t *R, bool act, int h, int n_i,
                                        uint64_t popm, uint32_t nzh, FitAdd fit_add,
                                        uint32_t &n_eval, uint32_t &n_acc, uint64_t &accm,
                                        int pt = 0) {
    static_assert(PARTS == 1 || PARTS == 2 || PARTS == 4, "parts");
    constexpr int SP = 32 / PARTS;  // solutions of the half per part
    int nm = 0, nd = 0;
    int u[M];
    uint64_t pw[M];
    uint32_t oh[M];
    if (act) {
        const int4 h0 = reinterpret_cast<const int4 *>(R)[0];
        const int4 h1 = reinterpret_cast<const int4 *>(R)[1];
        const int4 h2 = reinterpret_cast<const int4 *>(R)[2];
        const int4 h3 = reinterpret_cast<const int4 *>(R)[3];
        nm = h0.x;
        nd = h0.y;
        const int mem[kSmallSet] = {h0.z, h0.w, h1.x, h1.y, h1.z, h1.w, h2.x,
                                    h2.y, h2.z, h2.w, h3.x, h3.y, h3.z, h3.w};
#pragma unroll
        for (int k = 0; k < M; ++k) u[k] = k < nm ? mem[k] : -1;
    } else {
#pragma unroll
        for (int k = 0; k < M; ++k) u[k] = -1;
    }
    const uint32_t *O32 = reinterpret_cast<const uint32_t *>(O);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        pw[k] = u[k] >= 0 ? P[u[k]] : 0ull;
        oh[k] = u[k] >= 0 ? O32[2 * (size_t)u[k] + h] : 0u;
    }
    const uint16_t *rb = reinterpret_cast<const uint16_t *>(&L.rnd[tid >> 3][0]) + (tid & 7);
    // donors and change masks, one solution at a time
    uint32_t F[M];
#pragma unroll
    for (int k = 0; k < M; ++k) F[k] = 0u;
    uint32_t has = 0u;
    const int ii_lo = SP * pt;
    const int ii_hi = min(n_i, SP * pt + SP);
#pragma unroll 2
    for (int ii = ii_lo; ii < ii_hi; ++ii) {
        const int i = 32 * h + ii;
        uint32_t dlo = 0u, dhi = 0u;
        uint32_t s[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            s[k] = (uint32_t)__builtin_amdgcn_sbfe((int)oh[k], ii, 1u);
            dlo |= (uint32_t)pw[k] ^ s[k];
            dhi |= (uint32_t)(pw[k] >> 32) ^ s[k];
        }
        const uint64_t cand = popm & ~(1ull << i);
        dlo &= (uint32_t)cand;
        dhi &= (uint32_t)(cand >> 32);
        const uint32_t cnt = (uint32_t)__popc(dlo) + (uint32_t)__popc(dhi);
        const uint32_t h16 = rb[8 * ii];
        const uint32_t d = cnt ? select_bit(((uint64_t)dhi << 32) | dlo, (h16 * cnt) >> 16) : 0u;
        const uint32_t any = cnt ? 1u : 0u;
        has |= any << ii;
#pragma unroll
        for (int k = 0; k < M; ++k) F[k] |= ((bit_of(pw[k], d) ^ s[k]) & any) << ii;
    }
#pragma unroll
    for (int d = 8; d < 8 * PARTS; d <<= 1) {  // the partners' solutions' bits
#pragma unroll
        for (int k = 0; k < M; ++k) F[k] |= (uint32_t)__shfl_xor((int)F[k], d, 64);
        has |= (uint32_t)__shfl_xor((int)has, d, 64);
    }
    // fitness changes of the half's solutions, bit-sliced
#pragma unroll
    for (int k = 0; k < M; ++k) {
        L.fo[0][k][tid] = F[k];
        L.fo[1][k][tid] = oh[k];
    }
    uint32_t S[kGsPlanes], C[kGsPlanes];
#pragma unroll
    for (int j = 0; j < kGsPlanes; ++j) S[j] = C[j] = 0u;
    int32_t W = 0;
    // entries in batches of EB: the batch's record words, then its far-end words, are
    // requested before any is used (few waves share a SIMD, so each dependent round trip
    // would otherwise be paid in full)
    // (this lane's share of the entries)
    const int e_share = (nd + PARTS - 1) / PARTS;
    const int e_lo = min(nd, e_share * pt);
    const int e_hi = min(nd, e_lo + e_share);
    for (int e0 = e_lo; e0 < e_hi; e0 += EB) {
        int2 enb[EB];
        uint32_t ovb[EB];
#pragma unroll
        for (int q = 0; q < EB; ++q)  // past the share: inside, 0-0, weight 0
            enb[q] = e0 + q < e_hi ? reinterpret_cast<const int2 *>(R + 16)[e0 + q]
                                   : make_int2((int)0x80000000, 0);
#pragma unroll
        for (int q = 0; q < EB; ++q)
            ovb[q] = enb[q].x >= 0 ? O32[2 * (size_t)((uint32_t)enb[q].x & kSmallIdx) + h] : 0u;
#pragma unroll
        for (int q = 0; q < EB; ++q) {
            const int2 en = enb[q];
            const uint32_t x = (uint32_t)en.x;
            const int ka = (int)((x >> kSmallPosShift) & 15u);
            const uint32_t y = x & kSmallIdx;
            const bool inside = (int32_t)x < 0;
            const int kb = inside ? (int)y : ka;
            const uint32_t fa = L.fo[0][ka][tid], oa = L.fo[1][ka][tid];
            const uint32_t fb = L.fo[0][kb][tid], ob = L.fo[1][kb][tid];
            const uint32_t ov = inside ? ob : ovb[q];
            const uint32_t X = inside ? fa ^ fb : fa;
            const uint32_t cut = oa ^ ov;
            const uint32_t aw = (uint32_t)(en.y < 0 ? -en.y : en.y);
            const uint32_t A = X & (en.y > 0 ? ~cut : cut);
            const uint32_t nX = ~X;
            W += (int32_t)aw;
            // add |w| * (2 A + nX): plane j gets (A & bit j-1 of |w|) | (nX & bit j); a full
            // adder per plane, from the top so that C[j + 1] is read before plane j's carry
            // replaces it
            uint32_t wb[WB + 1];
#pragma unroll
            for (int j = 0; j < WB; ++j) wb[j] = (uint32_t)__builtin_amdgcn_sbfe((int)aw, j, 1u);
            wb[WB] = 0u;
#pragma unroll
            for (int j = kGsPlanes - 1; j >= 0; --j) {
                uint32_t z = 0u;
                if (j <= WB) z = (j ? A & wb[j - 1] : 0u) | (nX & wb[j]);
                const uint32_t sj = S[j], cj = C[j];
                S[j] = xor3(sj, cj, z);
                if (j + 1 < kGsPlanes) C[j + 1] = maj3(sj, cj, z);
            }
            C[0] = 0u;
        }
    }
#pragma unroll
    for (int d = 8; d < 8 * PARTS; d <<= 1) {  // add a partner's partial sum (two carry-save
        W += __shfl_xor(W, d, 64);             // additions per round)
        uint32_t XS[kGsPlanes], XC[kGsPlanes];  // (both read before either lane changes its own)
#pragma unroll
        for (int j = 0; j < kGsPlanes; ++j) {
            XS[j] = (uint32_t)__shfl_xor((int)S[j], d, 64);
            XC[j] = (uint32_t)__shfl_xor((int)C[j], d, 64);
        }
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int j = kGsPlanes - 1; j >= 0; --j) {
                const uint32_t sj = S[j], cj = C[j], xj = pass ? XC[j] : XS[j];
                S[j] = xor3(sj, cj, xj);
                if (j + 1 < kGsPlanes) C[j + 1] = maj3(sj, cj, xj);
            }
            C[0] = 0u;
        }
    }
    // T = S + C against W: greater / equal, all solutions at once
    uint32_t T[kGsPlanes];
    uint32_t carry = 0u;
#pragma unroll
    for (int j = 0; j < kGsPlanes; ++j) {
        T[j] = xor3(S[j], C[j], carry);
        carry = maj3(S[j], C[j], carry);
    }
    uint32_t gt = 0u, eq = ~0u;
#pragma unroll
    for (int j = kGsPlanes - 1; j >= 0; --j) {
        const uint32_t wj = (uint32_t)__builtin_amdgcn_sbfe(W, j, 1u);
        gt |= eq & T[j] & ~wj;
        eq &= ~(T[j] ^ wj);
    }
    const uint32_t acc = has & (gt | (eq & nzh));
    uint32_t *W32 = reinterpret_cast<uint32_t *>(O);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint32_t m = F[k] & acc;
        if (k % PARTS == pt && u[k] >= 0 && m) W32[2 * (size_t)u[k] + h] = oh[k] ^ m;
    }
    const uint32_t mine = PARTS == 1 ? acc : acc & (((1u << SP) - 1u) << (SP * pt));
    for (uint32_t m = mine; m; m &= m - 1) {
        const int ii = __builtin_ctz(m);
        int32_t t = 0;
#pragma unroll
        for (int j = 0; j < kGsPlanes; ++j) t |= (int32_t)((T[j] >> ii) & 1u) << j;
        fit_add(ii, (int64_t)(t - W));
    }
    if (pt == 0) {
        n_eval += (uint32_t)__popc(has);
        n_acc += (uint32_t)__popc(acc);
        accm |= (uint64_t)acc << (32 * h);
    }
}

// One colour class (per-class launch).  Blocks stride over tiles of kGsThreads slots.
template <int M, int WB>
__global__ __launch_bounds__(kGsThreads) void k_gen_swar_sweep(SweepArgs a) {
    static_assert(M >= 1 && M <= kSmallSet && WB >= 1 && WB + 1 < kGsPlanes, "shape");
    __shared__ GsLds<M, WB> L;
    __shared__ unsigned long long fa[64];
    __shared__ uint32_t redc[2][kGsThreads / 64];
    const int tid = (int)threadIdx.x;
    const uint64_t mism = a.stripes[tid & 63].mism;
    const bool live = a.st->elite_fitness < a.target;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t nz = a.always ? popm : (wave_or64(mism) & popm);
    if (tid < 64) fa[tid] = 0;
    __syncthreads();
    uint32_t n_eval = 0, n_acc = 0;
    uint64_t accm = 0;  // solutions with an accepted step (tracking mode)
    const int halves = a.N > 32 ? 2 : 1;
    const int slots = gs_slots(a.csize, halves);
    for (int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
         live && tile * kGsThreads < slots; tile += gridDim.x) {
        const GsItem it = gs_item(tile * kGsThreads + tid, halves);
        const bool act = it.p < a.csize;
        const int32_t *R = !act ? nullptr
                           : a.rstride ? a.recs + a.rbase + it.p * a.rstride
                                       : a.recs + a.roff[a.cbase + it.p];
        gs_draws(L.rnd, tid, a.seed, a.gen, a.cls, it.p, it.h);
        const int n_i = min(32, a.N - 32 * it.h);
        gs_step<M, WB, kGsEntryBatch>(L, tid, a.P, a.O, R, act, it.h, n_i, popm,
                                      (uint32_t)(nz >> (32 * it.h)),
                       [&](int ii, int64_t dl) {
                           atomicAdd(&fa[32 * it.h + ii], (unsigned long long)dl);
                       },
                       n_eval, n_acc, accm);
    }
    const uint32_t ce = wave_sum32(n_eval), ca = wave_sum32(n_acc);
    const uint64_t am = a.mode == kSweepGomTrack ? wave_or64(accm) : 0ull;
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) {
        redc[0][wave] = ce;
        redc[1][wave] = ca;
    }
    __syncthreads();
    Stripe *sp = a.stripes + (blockIdx.x % kStripes);
    if (tid < a.N && fa[tid])
        atomicAdd((unsigned long long *)&sp->fit[tid], fa[tid]);
    if (tid == 0) {
        uint32_t se = 0, sa = 0;
        for (int w = 0; w < kGsThreads / 64; ++w) {
            se += redc[0][w];
            sa += redc[1][w];
        }
        if (se) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)se);
        if (sa) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)sa);
    }
    if (lane == 0 && am) atomicOr((unsigned long long *)&sp->acc, (unsigned long long)am);
}

// Fused form: every class of the generation in one cooperative launch (all blocks resident at
// once, so a block may wait for others).  Block b sweeps chunk x = xcd_tile(b, grid) of each
// class in the generation's order.  Before a class it waits, one wave polling, until every
// chunk of an earlier class that holds a conflicting set carries this launch's stamp; after
// the class its threads' stores are made visible device-wide and the chunk is stamped.  A
// wait that polls kFusedSpinLimit times gives up and sets st->stall (the host reports it), so
// the kernel always ends.
template <bool PARTITION, bool NARROW>
__global__ __launch_bounds__(kSwarThreads) void k_uni_swar_fused(FusedArgs f) {
    using Acc = std::conditional_t<NARROW, int, unsigned long long>;
    const SweepArgs &a = f.a;
    const int x = xcd_tile((int)blockIdx.x, f.grid);
    const int lane = threadIdx.x & 63;
    const uint64_t mism = a.stripes[lane].mism;
    const bool live = a.st->elite_fitness < a.target;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t nz = a.always ? popm : (wave_or64(mism) & popm);
    __shared__ Acc fa[64];
    __shared__ uint32_t redc[2][kSwarThreads / 64];
    if (threadIdx.x < 64) fa[threadIdx.x] = 0;
    __syncthreads();
    if (!live) return;  // uniform over the grid
    uint32_t n_eval = 0, n_acc = 0;
    for (int t = 0; t < f.k; ++t) {
        const int c = f.order[t];
        const int lo = x * f.clen[c];
        const int hi = min(lo + f.clen[c], f.csize[c]);
        int p = lo + (int)threadIdx.x;
        // the chunk's first entries do not depend on other blocks: request them first
        SwarEntry en = swar_entry(a, f.cbase[c] + (p < hi ? p : 0));
        if (t > 0 && threadIdx.x < 64) {
            // wave 0 polls the flags of the earlier classes' chunks this chunk depends on,
            // lane l taking every 64th of them
            const int4 *dep = f.dep + ((size_t)c * f.grid + x) * f.k;
            uint32_t polls = 0;
            bool gave_up = false;
            for (int t2 = 0; t2 < t && !gave_up; ++t2) {
                const int c2 = f.order[t2];
                const int4 r4 = dep[c2];
                for (int h = 0; h < 2 && !gave_up; ++h) {
                    const int lo = h ? r4.z : r4.x, hi = h ? r4.w : r4.y;
                    // an unused range ({0, -1}) or one outside [0, grid) indexes no flag
                    if (lo < 0 || hi >= f.grid || lo > hi) continue;
                    for (int y = lo + lane; y <= hi && !gave_up; y += 64) {
                        uint32_t *fl = f.flags + (size_t)c2 * f.grid + y;
                        while (__hip_atomic_load(fl, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT) != f.epoch) {
                            if (++polls >= kFusedSpinLimit) {
                                gave_up = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(2);
                        }
                    }
                }
            }
            if (gave_up) atomicOr(const_cast<uint32_t *>(&a.st->stall), 1u);
            __threadfence();  // the chunks' stores are visible to this block's loads
        }
        __syncthreads();
        for (; p < hi; p += kSwarThreads) {
            if (p != lo + (int)threadIdx.x) en = swar_entry(a, f.cbase[c] + p);
            swar_step<PARTITION>(a, en, f.cbase[c] + p, popm, nz, fa, n_eval, n_acc);
        }
        __syncthreads();  // every store of the chunk is issued
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(f.flags + (size_t)c * f.grid + x, f.epoch, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    swar_block_totals(a, fa, redc, n_eval, n_acc);
}

// ------------------------------------------------------------------------------------------
// Resident schedule: one block per solution i runs all colour classes of one generation.
// The solution's offspring O_i lives in LDS, one byte per vertex; lane = set.  Per class:
// the block draws the Philox calls of the class once (thread t draws chunk t: the fields of
// 8 consecutive class positions), then every thread takes class positions t, t + 1024, ...
// and runs the GOM step for (i, set) exactly as the class-launch kernel does, reading the
// donors' genes from the population words P[u] and O_i from LDS.  Sets of one class never
// touch each other's variables or neighbours, so their byte updates do not race; a block
// barrier separates classes.  At the end the block packs O_i into a bit row (one ballot per
// 64 vertices) and adds its fitness change and counts to its stripe.
// ------------------------------------------------------------------------------------------
// LDS of a resident block of T threads: T Philox results (16 bytes each), the reduction
// area, the optional P copy, then the offspring bytes.
__host__ __device__ constexpr int res_rng_bytes(int T) { return T * 16; }
constexpr int kResRedBytes = 272;  // 16 wave sums (int64), 32 counts, 2 flags, padding

// LDS bytes of the P copy (16-byte multiple).
__host__ __device__ __forceinline__ size_t resident_words_bytes(int n) {
    return ((size_t)n * 8 + 15) & ~(size_t)15;
}

struct LdsCommit {
    uint8_t *ob;
    __device__ __forceinline__ void operator()(int u, bool flip) const {
        if (flip) ob[u] ^= 1u;
    }
};

// PLDS: the block also copies the population words P into LDS (8 bytes per vertex), so the
// donors' genes are read from LDS instead of global memory.
template <int KIND, bool PLDS, int T>
__device__ __forceinline__ void resident_body(const ResidentCtx &a, const uint16_t *order,
                                              int gen, int i, uint8_t *lds) {
    constexpr int kResRngBytes = res_rng_bytes(T);
    const uint64_t mism = a.stripes[threadIdx.x & 63].mism;
    if (a.st->elite_fitness >= a.target) return;
    uint32_t(*rng)[4] = reinterpret_cast<uint32_t(*)[4]>(lds);
    int64_t *redf = reinterpret_cast<int64_t *>(lds + kResRngBytes);
    uint32_t *redc = reinterpret_cast<uint32_t *>(lds + kResRngBytes + 128);
    uint64_t *pl = reinterpret_cast<uint64_t *>(lds + kResRngBytes + kResRedBytes);
    uint8_t *ob = lds + kResRngBytes + kResRedBytes + (PLDS ? resident_words_bytes(a.n) : 0);
    const uint64_t *P = PLDS ? pl : a.P;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t cand = popm & ~(1ull << i);
    const bool neutral_ok = a.always || bit_of(wave_or64(mism), (uint32_t)i);

    for (int v = tid; v < a.n; v += T) {
        const uint64_t w = a.P[v];
        if constexpr (PLDS) pl[v] = w;
        ob[v] = (uint8_t)bit_of(w, (uint32_t)i);
    }
    __syncthreads();

    const LdsBits bits{ob};
    const LdsCommit commit{ob};
    int64_t facc = 0;
    uint32_t n_eval = 0, n_acc = 0;
    for (int t = 0; t < a.k; ++t) {
        const int c = order[t];
        const int cbase = a.class_ptr[c];
        const int csize = a.class_ptr[c + 1] - cbase;
        const int2 cr = a.class_rec[c];  // {first record word, record stride or 0}
        auto record = [&](int p) {
            return AosRec{cr.y ? a.recs + cr.x + p * cr.y : a.recs + a.roff[cbase + p]};
        };
        for (int base = 0; base < csize; base += 8 * T) {
            const int span = min(csize - base, 8 * T);
            // issue this thread's first record of the round before the draws and the barrier
            AosRec R = record(base + (tid < span ? tid : 0));
            Head hd = load_head<KIND>(R);
            if constexpr (KIND != 0) {
                if (tid < ((span + 7) >> 3)) {
                    const U32x4 r = philox(a.seed, (uint32_t)gen, (uint32_t)c, (uint32_t)i,
                                           (uint32_t)((base >> 3) + tid));
                    rng[tid][0] = r.x;
                    rng[tid][1] = r.y;
                    rng[tid][2] = r.z;
                    rng[tid][3] = r.w;
                }
                __syncthreads();
            }
            for (int q = tid; q < span; q += T) {
                uint32_t h = 0;
                if constexpr (KIND != 0) {
                    const int f = q & 7;
                    h = (rng[q >> 3][f >> 1] >> (16 * (f & 1))) & 0xFFFFu;
                }
                if (q != tid) {
                    R = record(base + q);
                    hd = load_head<KIND>(R);
                }
                const PairOut r = gom_pair<KIND>(R, hd, P, bits, commit, cand, h, neutral_ok);
                facc += r.acc ? r.delta : 0;
                n_eval += r.cnt > 0;
                n_acc += r.acc;
            }
            __syncthreads();
        }
    }

    // forced improvement when no GOM step of this solution was accepted: the classes again,
    // in the same order, with the elitist as donor, until a class raises the fitness
    bool any_acc = false, improved = false;
    if (a.fi) {
        uint32_t *flags = redc + 32;  // [0]: accepted steps, [1]: an improving step
        if (tid == 0) flags[0] = flags[1] = 0u;
        __syncthreads();
        if (n_acc) atomicOr(&flags[0], 1u);
        __syncthreads();
        any_acc = flags[0] != 0u;
        const EliteWords ew{a.E};
        for (int t = 0; t < a.k && !any_acc && !improved; ++t) {
            const int c = order[t];
            const int cbase = a.class_ptr[c];
            const int csize = a.class_ptr[c + 1] - cbase;
            const int2 cr = a.class_rec[c];
            for (int q = tid; q < csize; q += T) {
                const AosRec R{cr.y ? a.recs + cr.x + q * cr.y : a.recs + a.roff[cbase + q]};
                const Head hd = load_head<KIND>(R);
                const PairOut r = gom_pair<KIND>(R, hd, ew, bits, commit, ~0ull, 0u, neutral_ok);
                facc += r.acc ? r.delta : 0;
                n_eval += r.cnt > 0;
                n_acc += r.acc;
                if (r.acc && r.delta > 0) atomicOr(&flags[1], 1u);
            }
            __syncthreads();
            improved = flags[1] != 0u;
        }
    }

    for (int v0 = wave * 64; v0 < a.n; v0 += T) {
        const int v = v0 + lane;
        const uint64_t word = ballot64(v < a.n && ob[v] != 0);
        if (lane == 0) a.rows[(size_t)i * a.row_words + (v0 >> 6)] = word;
    }
    facc = wave_sum64(facc);
    const uint32_t ce = wave_sum32(n_eval), ca = wave_sum32(n_acc);
    if (lane == 0) {
        redf[wave] = facc;
        redc[wave] = ce;
        redc[16 + wave] = ca;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t sf = 0;
        uint32_t se = 0, sa = 0;
        for (int w = 0; w < T / 64; ++w) {
            sf += redf[w];
            se += redc[w];
            sa += redc[16 + w];
        }
        Stripe *sp = a.stripes + (i % kStripes);
        if (sf) atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)sf);
        if (se) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)se);
        if (sa) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)sa);
        if (any_acc) atomicOr((unsigned long long *)&sp->acc, 1ull << i);
        if (improved) a.fi_at[i] = kFiBase;  // one block per solution: any nonzero record
    }
}

template <int KIND, bool PLDS>
__global__ __launch_bounds__(kResidentThreads) void k_resident_sweep(ResidentArgs a) {
    extern __shared__ __align__(16) uint8_t lds[];
    resident_body<KIND, PLDS, kResidentThreads>(a.c, a.order, a.c.gen, blockIdx.x, lds);
}

// ------------------------------------------------------------------------------------------
// Generation end (Algorithm 3: P <- O; the elitist is kept across generations), part 1, one
// wave: fitness of solution t = previous fitness + the stripes' changes; counters; best
// solution b (lowest index on ties); the elitist becomes P_b when f_b is strictly better
// (modes 0, 3, 4), always (mode 1, initial population) or never (mode 2).  In mode 4 (end
// of an iterated-local-search round) a solution whose change is negative keeps its previous
// fitness and is marked to keep its P genes.  Clears the stripes.  A generation skipped
// because the target was reached leaves everything as it is.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void finalize_body(const EpilogueArgs &a) {
    DevState *st = a.st;
    const int t = threadIdx.x;
    // every load is issued before the first wait: one round trip
    int64_t d = 0;
#pragma unroll
    for (int s = 0; s < kStripes; ++s) d += a.stripes[s].fit[t];
    const int64_t fit_t = a.fit[t];
    const uint64_t s_ev = a.stripes[t].evaluated, s_ac = a.stripes[t].accepted;
    const uint64_t s_acc = a.stripes[t].acc;
    const uint32_t fi_at = st->fi_at[t];
    const int64_t fE = st->elite_fitness;
    if (a.mode == kEpiGeneration && fE >= a.target) {
        if (t == 0) st->active = 0;
        return;
    }
    // forced improvement: the solutions it ran for and did not improve become the elitist
    uint64_t fail = 0;
    if (a.fi && a.mode == kEpiGeneration) {
        const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
        fail = popm & ~wave_or64(s_acc) & ~ballot64(fi_at != 0u);
    }
    // iterated local search: a solution whose round lowered its fitness keeps P
    const uint64_t rej = a.mode == kEpiIterated ? ballot64(t < a.N && d < 0) : 0ull;
    int64_t f = INT64_MIN;
    if (t < a.N) {
        f = bit_of(fail, (uint32_t)t) ? fE : bit_of(rej, (uint32_t)t) ? fit_t : fit_t + d;
        a.fit[t] = f;
    }
    const int64_t ev = wave_sum64((int64_t)s_ev);
    const int64_t ac = wave_sum64((int64_t)s_ac);
    int64_t fb = f;
    int b = t;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t of = __shfl_xor(fb, off, 64);
        const int ob = __shfl_xor(b, off, 64);
        if (of > fb || (of == fb && ob < b)) {
            fb = of;
            b = ob;
        }
    }
    __syncthreads();
#pragma unroll 16
    for (int s = 0; s < kStripes; ++s) a.stripes[s].fit[t] = 0;
    a.stripes[t].evaluated = 0;
    a.stripes[t].accepted = 0;
    a.stripes[t].mism = 0;
    a.stripes[t].acc = 0;
    st->fi_at[t] = 0u;
    if (t == 0) {
        st->fi_fail = fail;
        st->ils_rej = rej;
        const bool newE = a.mode == kEpiInit ||
                      ((a.mode == kEpiGeneration || a.mode == kEpiLocalSearch ||
                        a.mode == kEpiIterated) && fb > fE);
        st->best = b;
        st->new_elite = newE ? 1 : 0;
        st->active = 1;
        if (newE) st->elite_fitness = fb;
        if (a.mode == kEpiGeneration) st->generation += 1;
        st->evaluated += ev;
        st->accepted += ac;
        if (newE && fb >= a.target && st->done_tick < 0) st->done_tick = (int64_t)wall_clock64();
    }
}

__global__ __launch_bounds__(64) void k_finalize(EpilogueArgs a) { finalize_body(a); }

// ------------------------------------------------------------------------------------------
// Generation end, part 2, one thread per vertex: P <- O (modes 0 and 3; from the O planes,
// or from the solutions' bit rows under the resident schedule, then O is refreshed too; in
// mode 4 the solutions marked by the finalize take P back into O instead), the elitist
// bits (rewritten from P_b when the elitist changed), and the solutions whose genes differ
// from the elitist, OR-ed per block into the block's stripe.  The next generation's sweeps
// read those stripes to know which solutions equal the elitist.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void vertex_body(const EpilogueArgs &a, int vblock) {
    const DevState *st = a.st;
    const int tid = threadIdx.x, lane = tid & 63;
    const int v = vblock * kEpiThreads + tid;
    const bool in = v < a.n;
    // the vertex's words are loaded together with the run scalars (no wait in between)
    const uint64_t o_plane = a.O[in ? v : 0];
    const uint64_t e_word = a.E[(in ? v : 0) >> 6];
    if (!st->active) return;
    const int b = st->best;
    const bool newE = st->new_elite != 0;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    uint64_t o = 0ull;
    if (a.rows) {
        // lane t loads solution t's row word for this wave's 64 vertices; 64 ballots
        // transpose the 64 x 64 bit block so lane k ends with vertex k's word
        const int wv = (vblock * kEpiThreads + (tid & ~63)) >> 6;
        const uint64_t word =
            (lane < a.N && wv < a.row_words) ? a.rows[(size_t)lane * a.row_words + wv] : 0ull;
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            const uint64_t m = ballot64((word >> k) & 1ull);
            if (lane == k) o = m;
        }
        if (!in) o = 0ull;
    } else if (in) {
        o = o_plane;
    }
    if ((a.mode == kEpiGeneration || a.mode == kEpiLocalSearch) && in) {
        const uint64_t fail = st->fi_fail;
        if (fail) {  // copies of the elitist (its bits before this generation's update)
            const uint64_t eo = 0ull - (uint64_t)bit_of(e_word, (uint32_t)(v & 63));
            o = (o & ~fail) | (eo & fail);
        }
        a.P[v] = o;
        if (a.rows || fail) a.O[v] = o;
    } else if (a.mode == kEpiIterated && in) {
        const uint64_t rej = st->ils_rej;
        if (rej) {  // solutions that return to P
            o = (o & ~rej) | (a.P[v] & rej);
            a.O[v] = o;
        }
        a.P[v] = o;
    }
    uint32_t eb;
    if (newE) {
        eb = in ? bit_of(o, (uint32_t)b) : 0u;
        const uint64_t word = ballot64(eb != 0);
        if (lane == 0 && in) a.E[v >> 6] = word;
    } else {
        eb = in ? bit_of(e_word, (uint32_t)(v & 63)) : 0u;
    }
    const uint64_t mism = wave_or64(in ? ((o ^ (0ull - (uint64_t)eb)) & popm) : 0ull);
    __shared__ uint64_t sm[kEpiThreads / 64];
    if (lane == 0) sm[tid >> 6] = mism;
    __syncthreads();
    if (tid == 0) {
        uint64_t mm = 0;
#pragma unroll
        for (int w = 0; w < kEpiThreads / 64; ++w) mm |= sm[w];
        if (mm)
            atomicOr((unsigned long long *)&a.stripes[vblock % kStripes].mism,
                     (unsigned long long)mm);
    }
}

__global__ __launch_bounds__(kEpiThreads) void k_vertex_pass(EpilogueArgs a) {
    vertex_body(a, blockIdx.x);
}

// ------------------------------------------------------------------------------------------
// Batched generation step.  The sweep block for (instance b, solution i) first draws the
// instance's class order for its current generation (Fisher-Yates with the order stream:
// the draws in parallel, the swaps by one thread), then runs the resident sweep.  The
// finalize and vertex-pass blocks find their instance through the block maps.
// ------------------------------------------------------------------------------------------
// KIND: the FOS kind of every instance of the launch (univariate records take far fewer
// registers, so their blocks fill a CU twice as densely).
template <int T, int KIND>
__global__ __launch_bounds__(T) void k_batch_sweep(const BatchInst *insts, const int2 *blk) {
    extern __shared__ __align__(16) uint8_t lds_all[];
    uint16_t *order = reinterpret_cast<uint16_t *>(lds_all);
    uint16_t *draw = order + kResidentMaxClasses;
    const int2 bi = blk[blockIdx.x];
    const BatchInst *I = insts + bi.x;
    const ResidentCtx a = I->res;
    if (a.st->elite_fitness >= a.target) return;
    const int gen = a.st->generation;
    const bool fixed = I->order_fixed != 0;
    for (int t = threadIdx.x; t < a.k; t += T) {
        order[t] = (uint16_t)t;
        if (!fixed && t >= 1) {
            const U32x4 r = philox(a.seed, (uint32_t)gen, kOrderStream, (uint32_t)t, 0u);
            draw[t] = (uint16_t)(((uint64_t)r.x * (uint64_t)(t + 1)) >> 32);
        }
    }
    __syncthreads();
    if (!fixed && threadIdx.x == 0)
        for (int t = a.k - 1; t >= 1; --t) {
            const uint16_t x = order[t];
            order[t] = order[draw[t]];
            order[draw[t]] = x;
        }
    __syncthreads();
    uint8_t *lds = lds_all + kBatchOrderBytes;
    if (I->plds)
        resident_body<KIND, true, T>(a, order, gen, bi.y, lds);
    else
        resident_body<KIND, false, T>(a, order, gen, bi.y, lds);
}

__global__ __launch_bounds__(64) void k_batch_finalize(const BatchInst *insts) {
    if (insts[blockIdx.x].solo) return;  // its own epilogue runs with its sweeps
    finalize_body(insts[blockIdx.x].epi);
}

__global__ __launch_bounds__(kEpiThreads) void k_batch_vertex(const BatchInst *insts,
                                                              const int32_t *vblk) {
    const BatchInst *I = insts + vblk[blockIdx.x];
    vertex_body(I->epi, (int)blockIdx.x - I->vblock0);
}

// ------------------------------------------------------------------------------------------
// Batched class launch.  Planning, part 1 (one block per instance): the instance's class order
// of its current generation, the same Fisher-Yates draws as the host and the batched resident
// sweep.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bcl_order(const BclInst *insts, uint16_t *order,
                                                   int kmax, uint64_t *nzm) {
    __shared__ uint16_t draw[2048];
    const BclInst &I = insts[blockIdx.x];
    uint16_t *ord = order + (size_t)blockIdx.x * kmax;
    const int gen = I.st->generation;
    const bool fixed = I.order_fixed != 0;
    if (nzm && threadIdx.x < 64) {  // (wave 0, every lane) the neutral-step mask
        const uint64_t popm = I.N >= 64 ? ~0ull : ((1ull << I.N) - 1ull);
        const uint64_t m = wave_or64(I.stripes[threadIdx.x].mism);
        if (threadIdx.x == 0) nzm[blockIdx.x] = I.always ? popm : (m & popm);
    }
    for (int t = threadIdx.x; t < I.k; t += 256) {
        ord[t] = (uint16_t)t;
        if (!fixed && t >= 1) {
            const U32x4 r = philox(I.seed, (uint32_t)gen, kOrderStream, (uint32_t)t, 0u);
            draw[t] = (uint16_t)(((uint64_t)r.x * (uint64_t)(t + 1)) >> 32);
        }
    }
    __syncthreads();
    if (!fixed && threadIdx.x == 0)
        for (int t = I.k - 1; t >= 1; --t) {
            const uint16_t x = ord[t];
            ord[t] = ord[draw[t]];
            ord[draw[t]] = x;
        }
}

// Planning, part 2 (one block per position t): tiles of each instance's class at position t
// (none past its class count or once its target is reached), and their exclusive prefix sums
// over the instances; the total follows the last instance.
__global__ __launch_bounds__(256) void k_bcl_tiles(const BclInst *insts, const uint16_t *order,
                                                   int32_t *tiles, int count, int kmax,
                                                   int tile, int gs, int4 *pos) {
    __shared__ int32_t part[256];
    const int t = blockIdx.x;
    int32_t *row = tiles + (size_t)t * (count + 1);
    int32_t base = 0;
    for (int i0 = 0; i0 < count; i0 += 256) {
        const int i = i0 + (int)threadIdx.x;
        int32_t n = 0;
        if (i < count) {
            const BclInst &I = insts[i];
            if (t < I.k && I.st->elite_fitness < I.target) {
                const int c = order[(size_t)i * kmax + t];
                const int32_t c0 = I.class_ptr[c], cs = I.class_ptr[c + 1] - c0;
                n = !gs ? (cs + tile - 1) / tile
                    : I.uni ? gs_slots_uni(cs) : gs_slots_bcl(cs, I.N > 32 ? 2 : 1);
                if (gs) {  // the sweep's view of the class, one load away
                    const int2 cr = I.class_rec[c];
                    int4 *ps = pos + 2 * ((size_t)t * count + i);
                    ps[0] = make_int4(c, c0, cs, I.st->generation);
                    ps[1] = make_int4(cr.x, cr.y, 0, 0);
                }
            }
        }
        part[threadIdx.x] = n;
        __syncthreads();
        // inclusive scan of the 256 counts (Hillis-Steele)
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (i < count) row[i] = base + part[threadIdx.x] - n;
        base += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) row[count] = base;
}

// The sweep of position t: blocks stride over the position's tiles; a tile is kBclWaves x ppw
// consecutive class positions of one instance, wave w of the block takes ppw of them, lane =
// solution (as the class-launch sweep with groups of 64: the record is wave-uniform, one
// Philox call serves up to eight consecutive positions).  Fitness changes and counts go to the
// instance's stripe of the tile, after each tile.
constexpr int kBclRowLds = 1024;  // instances whose tile offsets a block keeps in LDS

// (about 60 VGPRs with the staged pair evaluation: eight waves per SIMD)
__global__ __launch_bounds__(kBclThreads) void k_bcl_sweep(BclPlan pl, int t) {
    __shared__ int32_t srow[kBclRowLds + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t *row = pl.tiles + (size_t)t * (pl.count + 1);
    // the position's tile offsets in LDS (for the instance search of every tile), when they fit
    const bool in_lds = pl.count <= kBclRowLds;
    if (in_lds)
        for (int q = threadIdx.x; q <= pl.count; q += kBclThreads) srow[q] = row[q];
    __syncthreads();
    const int32_t *rs = in_lds ? srow : row;
    const int32_t total = rs[pl.count];
    const uint32_t i = (uint32_t)lane;
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        // the instance of this tile: the last one whose first tile is <= tile
        int lo = 0, hi = pl.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rs[mid] <= tile) lo = mid;
            else hi = mid - 1;
        }
        const int b = __builtin_amdgcn_readfirstlane(lo);
        const BclInst &I = pl.insts[b];
        const int c = pl.order[(size_t)b * pl.kmax + t];
        const int cbase = I.class_ptr[c];
        const int csize = I.class_ptr[c + 1] - cbase;
        const int2 cr = I.class_rec[c];
        const int p0 = __builtin_amdgcn_readfirstlane((tile - rs[b]) * kBclWaves * pl.ppw +
                                                      wave * pl.ppw);
        if (p0 >= csize) continue;
        const uint64_t mism = I.stripes[lane].mism;
        const bool act = (int)i < I.N;
        const uint64_t popm = I.N >= 64 ? ~0ull : ((1ull << I.N) - 1ull);
        const uint64_t cand = act ? (popm & ~(1ull << i)) : 0ull;
        const bool neutral_ok = (I.always != 0) | (bit_of(wave_or64(mism), i) != 0);
        const int gen = I.st->generation;
        U32x4 q{0u, 0u, 0u, 0u};
        int64_t facc = 0;
        uint32_t n_eval = 0, n_acc = 0;
#pragma unroll 1
        for (int f = 0; f < pl.ppw; ++f) {
            const int p = p0 + f;
            if (p >= csize) break;
            // one call per eight positions (counter word 3 = p / 8)
            if (f == 0 || (p & 7) == 0)
                q = philox(I.seed, (uint32_t)gen, (uint32_t)c, i, (uint32_t)(p >> 3));
            const int32_t *rec = cr.y ? I.recs + cr.x + p * cr.y : I.recs + I.roff[cbase + p];
            const int fl = p & 7;  // (wave-uniform) field of the call
            const uint32_t w = (fl >> 1) == 0 ? q.x : (fl >> 1) == 1 ? q.y
                             : (fl >> 1) == 2 ? q.z : q.w;
            const uint32_t h = (w >> (16 * (fl & 1))) & 0xFFFFu;
            const PairOut r = staged_pair(rec, I.P, I.O, i, cand, h, neutral_ok);
            facc += r.acc ? r.delta : 0;
            n_eval += (uint32_t)__popcll(ballot64(r.cnt > 0));
            n_acc += (uint32_t)__popcll(ballot64(r.acc));
        }
        Stripe *sp = I.stripes + ((p0 >> 3) % kStripes);
        if (act && facc)
            atomicAdd((unsigned long long *)&sp->fit[i], (unsigned long long)facc);
        if (lane == 0) {
            if (n_eval) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)n_eval);
            if (n_acc) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)n_acc);
        }
    }
}

// Bit-sliced form of the batched class launch at position t: lane = slot over the slots of
// every instance's class pi_i[t] (gs_slots per instance, prefix sums in `tiles`), one or two
// a set as in k_gen_swar_sweep; a block's slots may span several instances (each lane finds
// its own), whose fitness changes and counts it gathers in LDS and adds to their stripes at
// the end.  Eight aligned slots always belong to one instance, position group and half.
template <int WB>
__global__ __launch_bounds__(kGsThreads) void k_bcl_gs_sweep(BclPlan pl, int t) {
    constexpr int M = kBclMaxMembers;
    constexpr int kWaves = kGsThreads / 64;
    __shared__ int32_t srow[kBclRowLds + 1];
    __shared__ GsLds<M, WB> L;
    __shared__ unsigned long long fa[kWaves][64];  // per wave: its instance's fitness changes
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t *row = pl.tiles + (size_t)t * (pl.count + 1);
    // the grid covers the most slots any position can have: blocks past this position's
    // slots end before touching LDS (uniform over the block)
    const int32_t total = row[pl.count];
    const int base = (int)blockIdx.x * kGsThreads;
    if (base >= total) return;
    const bool in_lds = pl.count <= kBclRowLds;
    if (in_lds)
        for (int q = tid; q <= pl.count; q += kGsThreads) srow[q] = row[q];
    fa[wave][lane] = 0ull;
    __syncthreads();
    const int32_t *rs = in_lds ? srow : row;
    // Every instance's slot count is a multiple of 64, so a wave's slots belong to one
    // instance (or all lie past the position's total): the last instance whose first slot is
    // <= the wave's first slot, found by a wave-uniform binary search
    const int q0 = base + 64 * wave, q = q0 + lane;
    const bool wave_ok = q0 < total;
    int lo = 0, hi = pl.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rs[mid] <= q0) lo = mid;
        else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const BclInst &I = pl.insts[b];
    const int4 pa = pl.pos[2 * ((size_t)t * pl.count + b)];
    const int4 pb = pl.pos[2 * ((size_t)t * pl.count + b) + 1];
    const int c = pa.x, cbase = pa.y, csize = pa.z, gen = pa.w;
    const uint64_t popm = I.N >= 64 ? ~0ull : ((1ull << I.N) - 1ull);
    uint32_t n_eval = 0, n_acc = 0;
    if (I.uni) {  // (wave-uniform) univariate: lane = set, all solutions in one word
        const int p = q - rs[b];
        if (wave_ok && p < csize) {
            SweepArgs a{};
            a.P = I.P;
            a.O = I.O;
            a.sw = I.sw;
            a.sw_stride = I.sw_stride;
            const SwarEntry en = swar_entry(a, cbase + p);
            if (I.partition)
                swar_step<true>(a, en, cbase + p, popm, pl.nzm[b], &fa[wave][0], n_eval, n_acc);
            else
                swar_step<false>(a, en, cbase + p, popm, pl.nzm[b], &fa[wave][0], n_eval, n_acc);
        }
    } else {
        const int halves = I.N > 32 ? 2 : 1;
        const GsItem2 it = gs_item2(q - rs[b], halves);
        const bool act = wave_ok && it.p < csize;
        const int32_t *R = !act ? nullptr
                           : pb.y ? I.recs + pb.x + it.p * pb.y : I.recs + I.roff[cbase + it.p];
        gs_draws<kGsPartsBcl>(L.rnd, tid, I.seed, gen, c, it.p, it.h, 32 / kGsPartsBcl * it.pt);
        uint64_t accm = 0;
        gs_step<M, WB, kGsEntryBatchBcl, kGsPartsBcl>(L, tid, I.P, I.O, R, act, it.h,
                                                      act ? min(32, I.N - 32 * it.h) : 0, popm,
                                                      (uint32_t)(pl.nzm[b] >> (32 * it.h)),
                                                      [&](int ii, int64_t dl) {
                                                          atomicAdd(&fa[wave][32 * it.h + ii],
                                                                    (unsigned long long)dl);
                                                      },
                                                      n_eval, n_acc, accm, it.pt);
    }
    const uint32_t ce = wave_sum32(n_eval), ca = wave_sum32(n_acc);
    __builtin_amdgcn_wave_barrier();
    if (!wave_ok) return;  // (uniform over the wave; no block barrier follows)
    Stripe *sp = I.stripes + ((int)blockIdx.x * kWaves + wave) % kStripes;
    const unsigned long long v = fa[wave][lane];
    if (v) atomicAdd((unsigned long long *)&sp->fit[lane], v);
    if (lane == 0) {
        if (ce) atomicAdd((unsigned long long *)&sp->evaluated, (unsigned long long)ce);
        if (ca) atomicAdd((unsigned long long *)&sp->accepted, (unsigned long long)ca);
    }
}

// Start of a batch run: every instance's start tick, and its done tick if the target is
// already reached.
__global__ void k_batch_mark(const BatchInst *insts, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    DevState *st = insts[t].epi.st;
    const int64_t now = (int64_t)wall_clock64();
    st->start_tick = now;
    st->done_tick = st->elite_fitness >= insts[t].epi.target ? now : -1;
}

// State hash terms of the genes (solution i, vertex v at byte i*n + v) and of the elitist
// bits (byte ebase + v); per-wave sums, one atomic add per wave (the sum is modulo 2^64, so the
// order of the adds does not change it).
__global__ __launch_bounds__(256) void k_state_hash(const uint64_t *X, const uint64_t *E, int n,
                                                   int N, uint64_t ebase, DevState *st) {
    const int v = blockIdx.x * 256 + threadIdx.x;
    uint64_t h = 0;
    if (v < n) {
        const uint64_t x = X[v];
        for (int i = 0; i < N; ++i)
            h += mix64((((uint64_t)i * (uint64_t)n + (uint64_t)v) << 8) | ((x >> i) & 1ull));
        const uint64_t e = (E[v >> 6] >> (v & 63)) & 1ull;
        h += mix64(((ebase + (uint64_t)v) << 8) | e);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)&st->hash, (unsigned long long)h);
}

__global__ void k_hash_zero(DevState *st) { st->hash = 0; }

__global__ void k_batch_gather(const BatchInst *insts, int count, DevState *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = *insts[t].epi.st;
}

}  // namespace

hipError_t launch_state_hash(const uint64_t *X, const uint64_t *E, int n, int N, uint64_t ebase,
                             DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_hash_zero, dim3(1), dim3(1), 0, s, st);
    hipLaunchKernelGGL(k_state_hash, dim3((n + 255) / 256), dim3(256), 0, s, X, E, n, N, ebase, st);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchInst *insts, int count, DevState *out, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_gather, dim3((count + 63) / 64), dim3(64), 0, s, insts, count, out);
    return hipGetLastError();
}

hipError_t launch_init_population(uint64_t *P, uint64_t *O, int64_t *fit, DevState *st,
                                  Stripe *stripes, int n, int N, uint64_t seed, hipStream_t s) {
    const int blocks128 = (n + 127) / 128;
    const int grid = (blocks128 + 3) / 4;
    hipLaunchKernelGGL(k_init_population, dim3(grid), dim3(256), 0, s, P, O, fit, st, stripes,
                       n, N, seed);
    return hipGetLastError();
}

hipError_t launch_zero_state(int64_t *fit, Stripe *stripes, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(256), 0, s, fit, stripes);
    return hipGetLastError();
}

hipError_t launch_full_fitness(const uint64_t *P, const int32_t *eu, const int32_t *ev,
                               const int32_t *ew, int64_t m, int N, Stripe *stripes,
                               hipStream_t s) {
    int64_t waves = (m + 15) / 16;
    int64_t grid = (waves + 3) / 4;
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_full_fitness, dim3((unsigned)grid), dim3(kFitThreads), 0, s, P, eu, ev,
                       ew, m, N, stripes);
    return hipGetLastError();
}

// Launch through hipExtLaunchKernelGGL when events are given: they take the dispatch's own
// start and end timestamps.
template <class K, class... Args>
static void launch_timed(K kernel, dim3 gd, dim3 bd, size_t lds, hipStream_t s, KernelEvents ev,
                         Args... args) {
    if (ev.start || ev.stop)
        hipExtLaunchKernelGGL(kernel, gd, bd, (uint32_t)lds, s, ev.start, ev.stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, gd, bd, lds, s, args...);
}

// Raise kernel K's dynamic LDS limit on the current device to at least `bytes`.  The limit is
// a per-device function attribute, so the largest size already set is kept per device; the
// check is lock-free and the update runs under a mutex, so host threads may launch at once.
constexpr int kMaxDevices = 64;

template <auto K>
static hipError_t raise_lds_limit(size_t bytes) {
    static std::atomic<size_t> done[kMaxDevices];
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (bytes <= done[dev].load(std::memory_order_acquire)) return hipSuccess;
    std::lock_guard<std::mutex> lock(mu);
    if (bytes <= done[dev].load(std::memory_order_relaxed)) return hipSuccess;
    e = hipFuncSetAttribute((const void *)K, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes);
    if (e == hipSuccess) done[dev].store(bytes, std::memory_order_release);
    return e;
}

// Static arena of gom_state_init_static: a state's device memory for callers that cannot
// allocate.  Each device holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is not a device address in
// host code).
static __device__ __align__(256) uint8_t scratch[kStaticArenaBytes];

hipError_t static_arena_address(void **ptr) {
    static void *addr[kMaxDevices] = {};
    static std::mutex mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_class_sweep_staged(const SweepArgs &a, int max_grid, int threads,
                                     hipStream_t s, KernelEvents ev) {
    if (threads < 64 || threads > kSweepMaxThreads || threads % 64) return hipErrorInvalidValue;
    const int wpb = threads / 64;
    const int64_t slots = (int64_t)max_grid * wpb;
    const bool shared = (int64_t)a.csize >= 8 * slots;
    const int per = shared ? 8 : 1;
    int grid = (int)std::min<int64_t>(max_grid, (a.csize + (int64_t)per * wpb - 1) /
                                                    ((int64_t)per * wpb));
    if (grid < 1) return hipSuccess;
    if (shared) launch_timed(k_class_sweep_staged<8>, dim3(grid), dim3(threads), 0, s, ev, a);
    else launch_timed(k_class_sweep_staged<1>, dim3(grid), dim3(threads), 0, s, ev, a);
    return hipGetLastError();
}

hipError_t launch_class_sweep(const SweepArgs &a, int kind, bool short_records, int max_grid,
                              int threads, hipStream_t s, KernelEvents ev) {
    if (threads < 64 || threads > kSweepMaxThreads || threads % 64) return hipErrorInvalidValue;
    const int G = a.N <= 16 ? 16 : (a.N <= 32 ? 32 : 64);
    const int per_tile = (threads / 64) * (64 / G);  // sets per block
    int grid = (a.csize + per_tile - 1) / per_tile;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) return hipSuccess;
    const dim3 gd(grid), bd(threads);
    // general records: share each Philox call over its eight positions when every group of
    // the largest grid would stride over at least eight positions anyway
    const int64_t slots = (int64_t)max_grid * per_tile;
    const bool shared = kind != 0 && a.mode != kSweepFi && (int64_t)a.csize >= 8 * slots;
    const int grid8 = (int)std::min<int64_t>(max_grid, (a.csize + 8 * per_tile - 1) /
                                                           (8 * (int64_t)per_tile));
    auto go = [&](auto fi) {
        constexpr bool FI = decltype(fi)::value;
        // several sets per wave (G < 64) read records with vector loads: no scalar registers
        // to save, so they keep the batch of 8
        if (kind == 0) {
            if (G == 16) launch_timed(k_class_sweep<16, 0, FI, 8>, gd, bd, 0, s, ev, a);
            else if (G == 32) launch_timed(k_class_sweep<32, 0, FI, 8>, gd, bd, 0, s, ev, a);
            else if (short_records) launch_timed(k_class_sweep<64, 0, FI, 4>, gd, bd, 0, s, ev, a);
            else launch_timed(k_class_sweep<64, 0, FI, 8>, gd, bd, 0, s, ev, a);
        } else if constexpr (!FI) {
            if (shared) {
                const dim3 gs(grid8);
                if (G == 16) launch_timed(k_class_sweep<16, 1, false, 8, 8>, gs, bd, 0, s, ev, a);
                else if (G == 32)
                    launch_timed(k_class_sweep<32, 1, false, 8, 8>, gs, bd, 0, s, ev, a);
                else if (short_records)
                    launch_timed(k_class_sweep<64, 1, false, 4, 8>, gs, bd, 0, s, ev, a);
                else launch_timed(k_class_sweep<64, 1, false, 8, 8>, gs, bd, 0, s, ev, a);
            } else {
                if (G == 16) launch_timed(k_class_sweep<16, 1, false, 8>, gd, bd, 0, s, ev, a);
                else if (G == 32) launch_timed(k_class_sweep<32, 1, false, 8>, gd, bd, 0, s, ev, a);
                else if (short_records)
                    launch_timed(k_class_sweep<64, 1, false, 4>, gd, bd, 0, s, ev, a);
                else launch_timed(k_class_sweep<64, 1, false, 8>, gd, bd, 0, s, ev, a);
            }
        } else {
            if (G == 16) launch_timed(k_class_sweep<16, 1, FI, 8>, gd, bd, 0, s, ev, a);
            else if (G == 32) launch_timed(k_class_sweep<32, 1, FI, 8>, gd, bd, 0, s, ev, a);
            else if (short_records) launch_timed(k_class_sweep<64, 1, FI, 4>, gd, bd, 0, s, ev, a);
            else launch_timed(k_class_sweep<64, 1, FI, 8>, gd, bd, 0, s, ev, a);
        }
    };
    if (a.mode == kSweepFi) go(std::true_type{});
    else go(std::false_type{});
    return hipGetLastError();
}

hipError_t launch_ls_sweep(const SweepArgs &a, int max_grid, hipStream_t s) {
    int grid = (a.csize + kLsThreads / 64 - 1) / (kLsThreads / 64);
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(k_ls_sweep, dim3(grid), dim3(kLsThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_perturb(const PerturbArgs &a, hipStream_t s) {
    if (a.flips < 1) return hipSuccess;
    if (a.flips > kPerturbMaxFlips || a.N < 1 || a.N > 64 || a.n_sets < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_perturb, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_split_sweep(const SweepArgs &a, hipStream_t s) {
    if (a.n_smap < 1) return hipSuccess;
    const dim3 gd(a.n_smap), bd(kSplitThreads);
    hipLaunchKernelGGL(k_split_donors, gd, bd, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_delta, gd, bd, 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_commit, gd, bd, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_large_set_sweep(const SweepArgs &a, int max_members, int threads,
                                  hipStream_t s) {
    if (a.n_large < 1) return hipSuccess;
    if (max_members < 1 || max_members > kCoopMaxMembers || a.coop_cap < max_members ||
        threads < 64 || threads > kCoopMaxThreads || threads % 64)
        return hipErrorInvalidValue;
    const size_t lds = 2 * sizeof(uint64_t) * (size_t)a.coop_cap;
    hipError_t e = raise_lds_limit<k_large_set_sweep>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_large_set_sweep, dim3(a.n_large), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_uni_swar_sweep(const SweepArgs &a, bool partition, bool narrow, int max_grid,
                                 hipStream_t s, KernelEvents ev) {
    int grid = (a.csize + kSwarThreads - 1) / kSwarThreads;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) return hipSuccess;
    const dim3 gd(grid), bd(kSwarThreads);
    if (partition && narrow) launch_timed(k_uni_swar_sweep<true, true>, gd, bd, 0, s, ev, a);
    else if (partition) launch_timed(k_uni_swar_sweep<true, false>, gd, bd, 0, s, ev, a);
    else if (narrow) launch_timed(k_uni_swar_sweep<false, true>, gd, bd, 0, s, ev, a);
    else launch_timed(k_uni_swar_sweep<false, false>, gd, bd, 0, s, ev, a);
    return hipGetLastError();
}

hipError_t launch_gen_swar_sweep(const SweepArgs &a, int members, int weight_bits, int max_grid,
                                 hipStream_t s, KernelEvents ev) {
    if (members < 1 || members > kGsMaxMembers || weight_bits < 1 ||
        weight_bits > kGsMaxWeightBits || a.N > 64)
        return hipErrorInvalidValue;
    int grid = (gs_slots(a.csize, a.N > 32 ? 2 : 1) + kGsThreads - 1) / kGsThreads;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) return hipSuccess;
    const dim3 gd(grid), bd(kGsThreads);
    if (members <= 5 && weight_bits <= 7) launch_timed(k_gen_swar_sweep<5, 7>, gd, bd, 0, s, ev, a);
    else if (members <= 5) launch_timed(k_gen_swar_sweep<5, 13>, gd, bd, 0, s, ev, a);
    else if (weight_bits <= 7) launch_timed(k_gen_swar_sweep<9, 7>, gd, bd, 0, s, ev, a);
    else launch_timed(k_gen_swar_sweep<9, 13>, gd, bd, 0, s, ev, a);
    return hipGetLastError();
}

hipError_t bcl_sweep_grid(int *grid) {
    int dev = 0, cus = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_bcl_sweep,
                                                         kBclThreads, 0);
    if (e != hipSuccess) return e;
    *grid = std::max(1, nb * cus);
    return hipSuccess;
}

hipError_t fused_swar_grid(int *grid) {
    int dev = 0, cus = 0, nb = 1 << 30;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *ks[4] = {(const void *)k_uni_swar_fused<true, true>,
                         (const void *)k_uni_swar_fused<true, false>,
                         (const void *)k_uni_swar_fused<false, true>,
                         (const void *)k_uni_swar_fused<false, false>};
    for (int q = 0; q < 4 && e == hipSuccess; ++q) {
        int b = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, ks[q], kSwarThreads, 0);
        nb = std::min(nb, b);
    }
    if (e != hipSuccess) return e;
    *grid = std::max(0, std::min(kFusedMaxGrid, nb * cus));
    return hipSuccess;
}

hipError_t launch_uni_swar_fused(const FusedArgs &f, bool partition, bool narrow,
                                 hipStream_t s) {
    if (f.grid < 1 || f.grid > kFusedMaxGrid || f.k < 1 || f.k > kFusedMaxClasses)
        return hipErrorInvalidValue;
    FusedArgs arg = f;
    void *args[] = {&arg};
    const void *k = partition ? (narrow ? (const void *)k_uni_swar_fused<true, true>
                                        : (const void *)k_uni_swar_fused<true, false>)
                              : (narrow ? (const void *)k_uni_swar_fused<false, true>
                                        : (const void *)k_uni_swar_fused<false, false>);
    return hipLaunchCooperativeKernel(k, dim3(f.grid), dim3(kSwarThreads), args, 0, s);
}

size_t resident_lds_bytes(int n, bool plds, int threads) {
    return (size_t)res_rng_bytes(threads) + kResRedBytes +
           (plds ? resident_words_bytes(n) : 0) + (((size_t)n + 15) & ~(size_t)15);
}

template <int KIND, bool PLDS>
static hipError_t launch_resident_t(const ResidentArgs &a, hipStream_t s, KernelEvents ev) {
    const size_t lds = resident_lds_bytes(a.c.n, PLDS, kResidentThreads);
    hipError_t e = raise_lds_limit<k_resident_sweep<KIND, PLDS>>(lds);
    if (e != hipSuccess) return e;
    launch_timed(k_resident_sweep<KIND, PLDS>, dim3(a.c.N), dim3(kResidentThreads), lds, s, ev,
                 a);
    return hipGetLastError();
}

hipError_t launch_resident_sweep(const ResidentArgs &a, int kind, bool plds, hipStream_t s,
                                 KernelEvents ev) {
    if (kind == 0)
        return plds ? launch_resident_t<0, true>(a, s, ev) : launch_resident_t<0, false>(a, s, ev);
    return plds ? launch_resident_t<1, true>(a, s, ev) : launch_resident_t<1, false>(a, s, ev);
}

// The batched sweep kernel of a launch group.
static const void *batch_kernel(int threads, int kind) {
    if (threads == 256)
        return kind == 0 ? (const void *)k_batch_sweep<256, 0> : (const void *)k_batch_sweep<256, 1>;
    return kind == 0 ? (const void *)k_batch_sweep<1024, 0> : (const void *)k_batch_sweep<1024, 1>;
}

hipError_t batch_sweep_occupancy(int threads, int kind, int *blocks) {
    if (threads != 256 && threads != 1024) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_kernel(threads, kind),
                                                        threads, 0);
}

hipError_t prepare_batch_step(const BatchLaunch *groups, int n_groups) {
    for (int q = 0; q < n_groups; ++q) {
        const BatchLaunch &G = groups[q];
        hipError_t e;
        if (G.threads == 256)
            e = G.kind == 0 ? raise_lds_limit<k_batch_sweep<256, 0>>(G.lds)
                            : raise_lds_limit<k_batch_sweep<256, 1>>(G.lds);
        else
            e = G.kind == 0 ? raise_lds_limit<k_batch_sweep<1024, 0>>(G.lds)
                            : raise_lds_limit<k_batch_sweep<1024, 1>>(G.lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch_step(const BatchInst *insts, int count, const int2 *blk,
                             const BatchLaunch *groups, int n_groups, const int32_t *vblk,
                             int vblocks, const BclPlan &bcl, hipStream_t s, KernelEvents ev) {
    hipError_t e = prepare_batch_step(groups, n_groups);
    if (e != hipSuccess) return e;
    // the step's timing spans the first sweep launch's start to the last one's end
    const int n_bcl = bcl.count > 0 ? bcl.kmax : 0;  // sweep launches of the class launches
    const int n_sweeps = n_groups + n_bcl;
    for (int q = 0; q < n_groups; ++q) {
        const BatchLaunch &G = groups[q];
        if (G.threads != 256 && G.threads != 1024) return hipErrorInvalidValue;
        KernelEvents gev;
        gev.start = q == 0 ? ev.start : nullptr;
        gev.stop = q == n_sweeps - 1 ? ev.stop : nullptr;
        const int2 *gb = blk + G.first;
        if (G.threads == 256 && G.kind == 0)
            launch_timed(k_batch_sweep<256, 0>, dim3(G.count), dim3(256), G.lds, s, gev, insts, gb);
        else if (G.threads == 256)
            launch_timed(k_batch_sweep<256, 1>, dim3(G.count), dim3(256), G.lds, s, gev, insts, gb);
        else if (G.kind == 0)
            launch_timed(k_batch_sweep<1024, 0>, dim3(G.count), dim3(1024), G.lds, s, gev, insts,
                         gb);
        else
            launch_timed(k_batch_sweep<1024, 1>, dim3(G.count), dim3(1024), G.lds, s, gev, insts,
                         gb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_bcl > 0) {
        if (bcl.kmax > 2048 || bcl.grid < 1) return hipErrorInvalidValue;
        if (bcl.gs && (!bcl.nzm || !bcl.pos || bcl.gs_grid < 1 ||
                       (bcl.gs_wb != 7 && bcl.gs_wb != 13)))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_bcl_order, dim3(bcl.count), dim3(256), 0, s, bcl.insts, bcl.order,
                           bcl.kmax, bcl.gs ? bcl.nzm : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (bcl.ppw < 1 || bcl.ppw > kBclPositions) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_bcl_tiles, dim3(bcl.kmax), dim3(256), 0, s, bcl.insts, bcl.order,
                           bcl.tiles, bcl.count, bcl.kmax, kBclWaves * bcl.ppw, bcl.gs, bcl.pos);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        for (int t = 0; t < bcl.kmax; ++t) {
            KernelEvents gev;
            gev.start = n_groups == 0 && t == 0 ? ev.start : nullptr;
            gev.stop = t == bcl.kmax - 1 ? ev.stop : nullptr;
            if (!bcl.gs)
                launch_timed(k_bcl_sweep, dim3(bcl.grid), dim3(kBclThreads), 0, s, gev, bcl, t);
            else if (bcl.gs_wb == 7)
                launch_timed(k_bcl_gs_sweep<7>, dim3(bcl.gs_grid), dim3(kGsThreads), 0, s, gev,
                             bcl, t);
            else
                launch_timed(k_bcl_gs_sweep<13>, dim3(bcl.gs_grid), dim3(kGsThreads), 0, s, gev,
                             bcl, t);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_batch_finalize, dim3(count), dim3(64), 0, s, insts);
    e = hipGetLastError();
    if (e != hipSuccess || vblocks < 1) return e;  // (a batch of solo instances only)
    hipLaunchKernelGGL(k_batch_vertex, dim3(vblocks), dim3(kEpiThreads), 0, s, insts, vblk);
    return hipGetLastError();
}

hipError_t launch_batch_mark(const BatchInst *insts, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_mark, dim3((count + 255) / 256), dim3(256), 0, s, insts, count);
    return hipGetLastError();
}

hipError_t launch_epilogue(const EpilogueArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = (a.n + kEpiThreads - 1) / kEpiThreads;
    hipLaunchKernelGGL(k_vertex_pass, dim3(grid), dim3(kEpiThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace gom
