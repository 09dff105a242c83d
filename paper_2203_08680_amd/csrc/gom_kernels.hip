// gom_kernels.hip -- CDNA4 (gfx950) kernels of libgom.
//
// Data layout in HBM (one state):
//   P, O   population at generation start and offspring, one 64-bit word per vertex; bit i of
//          word v is gene v of solution i (bit-planes: a vertex's genes for the whole
//          population, up to 64 solutions, travel in one 8-byte access).
//   E      elitist genes, bit (v mod 64) of word v / 64.
//   fit    int64 fitness per solution.
//   records of the FOS sets in colour-class order (see SweepArgs).
//
// A generation runs under one of two schedules with identical results:
//   class launch: one k_class_sweep launch per colour class (in the generation's class
//     order), lane = solution, offspring in the O planes;
//   resident:     one k_resident_sweep launch (block = solution, offspring in LDS, all
//     classes), offspring written back as one bit row per solution;
// then one k_epilogue launch (P <- O, elitist update, equality flags).  Integer arithmetic
// only, so every result is exact and independent of the order in which waves run.
#include "gom_internal.h"

namespace gom {
namespace {

constexpr int kSweepThreads = 512;  // 8 waves of 64 lanes
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

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x |= __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// ------------------------------------------------------------------------------------------
// Initial population (Algorithm 3, InitializePopulation): gene v of solution i is bit
// (v mod 32) of word ((v / 32) mod 4) of Philox(seed; kInitStream, i, v / 128, 0).
// One wave per 128 vertices: lane i draws solution i's 128 genes, then 128 ballots turn them
// into the 128 population words, two per lane, stored coalesced.  Block 0 also clears the
// fitness accumulators and the run scalars.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_population(uint64_t *P, uint64_t *O, int64_t *fit,
                                                         DevState *st, int n, int N,
                                                         uint64_t seed) {
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) fit[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            st->elite_fitness = INT64_MIN;
            st->eq = 0;
            st->mism = 0;
            st->evaluated = 0;
            st->accepted = 0;
            st->generation = 0;
            st->blocks_done = 0;
            st->best = 0;
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

__global__ void k_zero_state(int64_t *fit, DevState *st) {
    if (threadIdx.x < 64) fit[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        st->mism = 0;
        st->blocks_done = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Full Max-Cut fitness of every solution (Section 6.2): one wave per edge at a time, lane i
// adds the weight when bit i of P[u] xor P[v] is set (the edge is cut in solution i).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kFitThreads) void k_full_fitness(const uint64_t *P,
                                                              const int32_t *eu,
                                                              const int32_t *ev,
                                                              const int32_t *ew, int64_t m,
                                                              int N, int64_t *fit) {
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
        if (s) atomicAdd((unsigned long long *)&fit[threadIdx.x], (unsigned long long)s);
    }
}

// ------------------------------------------------------------------------------------------
// One colour class of one generation (Algorithm 3, the body of the loop over groups; the GOM
// step of Algorithm 2 for every (solution, set) pair of the class at once).
//
// Mapping: a group of G lanes (G = 16, 32 or 64, the population rounded up) takes one set of
// the class; lane i of the group is solution i.  A block of 8 waves takes a tile of
// 8 * 64 / G consecutive class positions.  All sets of one class are independent (no shared
// or adjacent variables), so groups never read a word that another group of the same launch
// writes, and each O word of a set is written by exactly one lane.
//
// Per pair (solution i, set F_j at class position p):
//   D      = solutions d != i whose P genes differ from O_i somewhere on F_j (64-bit mask,
//            OR over the members of (P[u] xor broadcast(O_i[u])))
//   h      = 16-bit field (p mod 8) of Philox(seed; g, c, i, p / 8); the block draws the 64
//            calls of a tile once (wave 0) and shares them through LDS
//   donor  = the r-th set bit of D with r = (h * |D|) >> 16
//   C      = members u where the donor's gene differs from O_i[u]
//   delta  = sum over the set's dependent edges of the change of the cut: an outside edge
//            (u, v) changes when u is in C, an inside edge when exactly one end is in C; the
//            change is +w if the edge was uncut, -w if it was cut
//   accept = |D| > 0 and (delta > 0 or (delta == 0 and (always or P_i != elitist)))
//   commit = one word store per member: O[u] ^= ballot(accept and u in C)
// A univariate FOS (every set one variable) needs no draw: the donor always differs at that
// variable, so C = {j} whenever D is non-empty, whichever donor is drawn.
// Fitness deltas are summed per block and added once per solution with an int64 atomic.
// ------------------------------------------------------------------------------------------
template <int G, bool UNI>
__global__ __launch_bounds__(kSweepThreads) void k_class_sweep(SweepArgs a) {
    if (a.st->elite_fitness >= a.target) return;
    const uint64_t eq = a.st->eq;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int GPW = 64 / G;          // sets per wave
    constexpr int PER_TILE = 8 * GPW;    // sets per block tile (multiple of 8)
    const int grp = lane / G;
    const uint32_t i = (uint32_t)(lane % G);
    const bool act = (int)i < a.N;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t cand = popm & ~(1ull << i);
    const bool neutral_ok = a.always || !bit_of(eq, i);

    __shared__ uint32_t rng[64][4];
    __shared__ int64_t red[kSweepThreads];
    __shared__ uint32_t redc[2][8];

    int64_t facc = 0;
    uint32_t n_eval = 0, n_acc = 0;
    const int ntiles = (a.csize + PER_TILE - 1) / PER_TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int base = tile * PER_TILE;
        if constexpr (!UNI) {
            if (wave == 0) {
                const int q = lane / G;
                const int p0 = base + q * 8;
                if (p0 < a.csize) {
                    const U32x4 r = philox(a.seed, (uint32_t)a.gen, (uint32_t)a.cls,
                                           (uint32_t)(lane % G), (uint32_t)(p0 >> 3));
                    rng[lane][0] = r.x;
                    rng[lane][1] = r.y;
                    rng[lane][2] = r.z;
                    rng[lane][3] = r.w;
                }
            }
            __syncthreads();
        }
        const int local = wave * GPW + grp;
        const int p = base + local;
        if (p < a.csize) {
            const int s = a.cbase + p;
            int m0, m1;
            if constexpr (UNI) {
                m0 = s;
                m1 = s + 1;
            } else {
                m0 = a.mptr[s];
                m1 = a.mptr[s + 1];
            }
            // Eligible donors.
            uint64_t D = 0;
            for (int m = m0; m < m1; ++m) {
                const int u = a.mem_v[m];
                D |= a.P[u] ^ (0ull - (uint64_t)bit_of(a.O[u], i));
            }
            D &= cand;
            const uint32_t cnt = act ? (uint32_t)__popcll(D) : 0u;
            uint32_t d = 0;
            if constexpr (!UNI) {
                const int f = local & 7;
                const uint32_t h = (rng[(local >> 3) * G + (int)i][f >> 1] >> (16 * (f & 1))) &
                                   0xFFFFu;
                if (cnt) d = select_bit(D, (h * cnt) >> 16);
            }
            // Partial evaluation.
            int64_t delta = 0;
            for (int m = m0; m < m1; ++m) {
                const int u = a.mem_v[m];
                const uint32_t oq = bit_of(a.O[u], i);
                uint32_t cq = 1u;
                if constexpr (!UNI) cq = bit_of(a.P[u], d) ^ oq;
                const int e1 = a.mem_dptr[m + 1];
                for (int e = a.mem_dptr[m]; e < e1; ++e) {
                    const int2 en = a.dep[e];
                    uint32_t flip, ov;
                    if (en.x >= 0) {
                        ov = bit_of(a.O[en.x], i);
                        flip = cq;
                    } else {
                        const int v = ~en.x;
                        ov = bit_of(a.O[v], i);
                        flip = cq ^ (bit_of(a.P[v], d) ^ ov);
                    }
                    const int32_t sw = (oq == ov) ? en.y : -en.y;
                    delta += flip ? sw : 0;
                }
            }
            const bool acc = cnt > 0 && (delta > 0 || (delta == 0 && neutral_ok));
            // Commit accepted steps: one word per member.
            for (int m = m0; m < m1; ++m) {
                const int u = a.mem_v[m];
                const uint64_t ow = a.O[u];
                uint32_t cq = 1u;
                if constexpr (!UNI) cq = bit_of(a.P[u], d) ^ bit_of(ow, i);
                uint64_t fm = ballot64(acc && cq);
                if constexpr (G < 64) fm = (fm >> (grp * G)) & ((1ull << G) - 1ull);
                if (fm != 0 && i == 0) a.O[u] = ow ^ fm;
            }
            facc += acc ? delta : 0;
            n_eval += cnt > 0;
            n_acc += acc;
        }
        if constexpr (!UNI) __syncthreads();
    }

    red[tid] = facc;
    const uint32_t ce = wave_sum32(n_eval), ca = wave_sum32(n_acc);
    if (lane == 0) {
        redc[0][wave] = ce;
        redc[1][wave] = ca;
    }
    __syncthreads();
    if (tid < G && tid < a.N) {
        int64_t sum = 0;
        for (int w = 0; w < 8; ++w)
#pragma unroll
            for (int g2 = 0; g2 < GPW; ++g2) sum += red[w * 64 + g2 * G + tid];
        if (sum) atomicAdd((unsigned long long *)&a.fit[tid], (unsigned long long)sum);
    }
    if (tid == 0) {
        uint32_t se = 0, sa = 0;
        for (int w = 0; w < 8; ++w) {
            se += redc[0][w];
            sa += redc[1][w];
        }
        DevState *st = const_cast<DevState *>(a.st);
        if (se) atomicAdd((unsigned long long *)&st->evaluated, (unsigned long long)se);
        if (sa) atomicAdd((unsigned long long *)&st->accepted, (unsigned long long)sa);
    }
}

// ------------------------------------------------------------------------------------------
// Generation epilogue (Algorithm 3, P <- O; elitist kept across generations).
//   best b = argmax fitness (lowest index on ties); the elitist becomes P_b when f_b is
//   strictly better (mode 0), unconditionally (mode 1, initial population) or never (mode 2).
//   Every block copies its vertices' words O -> P (mode 0), refreshes or reads the elitist
//   bits, and ORs the solutions that differ from the elitist; the last block to arrive turns
//   that into the equality flags used by the next generation and updates the scalars.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kEpiThreads) void k_epilogue(EpilogueArgs a) {
    DevState *st = a.st;
    const int64_t fE = st->elite_fitness;
    if (a.mode == kEpiGeneration && fE >= a.target) return;
    int b = 0;
    int64_t fb = a.fit[0];
    for (int t = 1; t < a.N; ++t) {
        const int64_t x = a.fit[t];
        if (x > fb) { fb = x; b = t; }
    }
    const bool newE = a.mode == kEpiInit || (a.mode == kEpiGeneration && fb > fE);
    const int tid = threadIdx.x, lane = tid & 63;
    const int v = blockIdx.x * kEpiThreads + tid;
    const bool in = v < a.n;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    uint64_t o = 0ull;
    if (in) {
        if (a.rows) {
            // resident schedule: gather bit v of every solution's row
            const size_t wv = (size_t)(v >> 6);
            const uint32_t sh = (uint32_t)(v & 63);
            for (int t = 0; t < a.N; ++t)
                o |= ((a.rows[(size_t)t * a.row_words + wv] >> sh) & 1ull) << t;
        } else {
            o = a.O[v];
        }
    }
    if (a.mode == kEpiGeneration && in) {
        a.P[v] = o;
        if (a.rows) a.O[v] = o;
    }
    uint32_t eb;
    if (newE) {
        eb = in ? bit_of(o, (uint32_t)b) : 0u;
        const uint64_t word = ballot64(eb != 0);
        if (lane == 0 && v < a.n) a.E[v >> 6] = word;
    } else {
        eb = in ? bit_of(a.E[v >> 6], (uint32_t)(v & 63)) : 0u;
    }
    uint64_t mism = in ? ((o ^ (0ull - (uint64_t)eb)) & popm) : 0ull;
    mism = wave_or64(mism);
    __shared__ uint64_t sm[kEpiThreads / 64];
    __shared__ int last;
    if (lane == 0) sm[tid >> 6] = mism;
    __syncthreads();
    if (tid == 0) {
        uint64_t mm = 0;
#pragma unroll
        for (int w = 0; w < kEpiThreads / 64; ++w) mm |= sm[w];
        if (mm) atomicOr((unsigned long long *)&st->mism, (unsigned long long)mm);
        __threadfence();
        const uint32_t prev = atomicAdd(&st->blocks_done, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (last && tid == 0) {
        __threadfence();
        const uint64_t all = atomicOr((unsigned long long *)&st->mism, 0ull);
        st->eq = ~all & popm;
        if (newE) st->elite_fitness = fb;
        st->best = b;
        if (a.mode == kEpiGeneration) st->generation += 1;
        st->mism = 0;
        st->blocks_done = 0;
    }
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
// 64 vertices), adds its fitness change to fit[i] and its counts to the run counters.
// ------------------------------------------------------------------------------------------
constexpr int kResRngBytes = kResidentChunkSlots * 16;
constexpr int kResRedBytes = 256;

template <bool UNI>
__global__ __launch_bounds__(kResidentThreads) void k_resident_sweep(ResidentArgs a) {
    DevState *st = a.st;
    if (st->elite_fitness >= a.target) return;
    extern __shared__ __align__(16) uint8_t lds[];
    uint32_t(*rng)[4] = reinterpret_cast<uint32_t(*)[4]>(lds);
    int64_t *redf = reinterpret_cast<int64_t *>(lds + kResRngBytes);
    uint32_t *redc = reinterpret_cast<uint32_t *>(lds + kResRngBytes + 128);
    uint8_t *ob = lds + kResRngBytes + kResRedBytes;

    const int i = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t popm = a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull);
    const uint64_t cand = popm & ~(1ull << i);
    const bool neutral_ok = a.always || !bit_of(st->eq, (uint32_t)i);

    for (int v = tid; v < a.n; v += kResidentThreads) ob[v] = (uint8_t)bit_of(a.P[v], (uint32_t)i);
    __syncthreads();

    int64_t facc = 0;
    uint32_t n_eval = 0, n_acc = 0;
    for (int t = 0; t < a.k; ++t) {
        const int c = a.order[t];
        const int cbase = a.class_ptr[c];
        const int csize = a.class_ptr[c + 1] - cbase;
        for (int base = 0; base < csize; base += 8 * kResidentChunkSlots) {
            const int span = min(csize - base, 8 * kResidentChunkSlots);
            if constexpr (!UNI) {
                if (tid < ((span + 7) >> 3)) {
                    const U32x4 r = philox(a.seed, (uint32_t)a.gen, (uint32_t)c, (uint32_t)i,
                                           (uint32_t)((base >> 3) + tid));
                    rng[tid][0] = r.x;
                    rng[tid][1] = r.y;
                    rng[tid][2] = r.z;
                    rng[tid][3] = r.w;
                }
                __syncthreads();
            }
            for (int q = tid; q < span; q += kResidentThreads) {
                const int s = cbase + base + q;
                int m0, m1;
                if constexpr (UNI) {
                    m0 = s;
                    m1 = s + 1;
                } else {
                    m0 = a.mptr[s];
                    m1 = a.mptr[s + 1];
                }
                uint64_t D = 0;
                for (int m = m0; m < m1; ++m) {
                    const int u = a.mem_v[m];
                    D |= a.P[u] ^ (0ull - (uint64_t)ob[u]);
                }
                D &= cand;
                const uint32_t cnt = (uint32_t)__popcll(D);
                if (cnt == 0) continue;
                uint32_t d = 0;
                if constexpr (!UNI) {
                    const int f = q & 7;
                    const uint32_t h = (rng[q >> 3][f >> 1] >> (16 * (f & 1))) & 0xFFFFu;
                    d = select_bit(D, (h * cnt) >> 16);
                }
                int64_t delta = 0;
                for (int m = m0; m < m1; ++m) {
                    const int u = a.mem_v[m];
                    const uint32_t oq = ob[u];
                    uint32_t cq = 1u;
                    if constexpr (!UNI) cq = bit_of(a.P[u], d) ^ oq;
                    const int e1 = a.mem_dptr[m + 1];
                    for (int e = a.mem_dptr[m]; e < e1; ++e) {
                        const int2 en = a.dep[e];
                        uint32_t flip, ov;
                        if (en.x >= 0) {
                            ov = ob[en.x];
                            flip = cq;
                        } else {
                            const int v = ~en.x;
                            ov = ob[v];
                            flip = cq ^ (bit_of(a.P[v], d) ^ ov);
                        }
                        const int32_t sw = (oq == ov) ? en.y : -en.y;
                        delta += flip ? sw : 0;
                    }
                }
                ++n_eval;
                if (delta > 0 || (delta == 0 && neutral_ok)) {
                    for (int m = m0; m < m1; ++m) {
                        const int u = a.mem_v[m];
                        if constexpr (UNI) {
                            ob[u] ^= 1u;
                        } else {
                            const uint32_t oq = ob[u];
                            if (bit_of(a.P[u], d) ^ oq) ob[u] = (uint8_t)(oq ^ 1u);
                        }
                    }
                    facc += delta;
                    ++n_acc;
                }
            }
            __syncthreads();
        }
    }

    for (int v0 = wave * 64; v0 < a.n; v0 += kResidentThreads) {
        const int v = v0 + lane;
        const uint64_t word = ballot64(v < a.n && ob[v] != 0);
        if (lane == 0) a.rows[(size_t)i * a.row_words + (v0 >> 6)] = word;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) facc += __shfl_xor(facc, off, 64);
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
        for (int w = 0; w < kResidentThreads / 64; ++w) {
            sf += redf[w];
            se += redc[w];
            sa += redc[16 + w];
        }
        a.fit[i] += sf;
        if (se) atomicAdd((unsigned long long *)&st->evaluated, (unsigned long long)se);
        if (sa) atomicAdd((unsigned long long *)&st->accepted, (unsigned long long)sa);
    }
}
}  // namespace

hipError_t launch_init_population(uint64_t *P, uint64_t *O, int64_t *fit, DevState *st, int n,
                                  int N, uint64_t seed, hipStream_t s) {
    const int blocks128 = (n + 127) / 128;
    const int grid = (blocks128 + 3) / 4;
    hipLaunchKernelGGL(k_init_population, dim3(grid), dim3(256), 0, s, P, O, fit, st, n, N, seed);
    return hipGetLastError();
}

hipError_t launch_zero_state(int64_t *fit, DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, s, fit, st);
    return hipGetLastError();
}

hipError_t launch_full_fitness(const uint64_t *P, const int32_t *eu, const int32_t *ev,
                               const int32_t *ew, int64_t m, int N, int64_t *fit, hipStream_t s) {
    int64_t waves = (m + 15) / 16;
    int64_t grid = (waves + 3) / 4;
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_full_fitness, dim3((unsigned)grid), dim3(kFitThreads), 0, s, P, eu, ev,
                       ew, m, N, fit);
    return hipGetLastError();
}

hipError_t launch_class_sweep(const SweepArgs &a, bool univariate, int max_grid, hipStream_t s) {
    const int G = a.N <= 16 ? 16 : (a.N <= 32 ? 32 : 64);
    const int per_tile = 8 * (64 / G);
    int grid = (a.csize + per_tile - 1) / per_tile;
    if (grid > max_grid) grid = max_grid;
    if (grid < 1) return hipSuccess;
    const dim3 gd(grid), bd(kSweepThreads);
    if (univariate) {
        if (G == 16) hipLaunchKernelGGL((k_class_sweep<16, true>), gd, bd, 0, s, a);
        else if (G == 32) hipLaunchKernelGGL((k_class_sweep<32, true>), gd, bd, 0, s, a);
        else hipLaunchKernelGGL((k_class_sweep<64, true>), gd, bd, 0, s, a);
    } else {
        if (G == 16) hipLaunchKernelGGL((k_class_sweep<16, false>), gd, bd, 0, s, a);
        else if (G == 32) hipLaunchKernelGGL((k_class_sweep<32, false>), gd, bd, 0, s, a);
        else hipLaunchKernelGGL((k_class_sweep<64, false>), gd, bd, 0, s, a);
    }
    return hipGetLastError();
}

size_t resident_lds_bytes(int n) {
    return (size_t)kResRngBytes + kResRedBytes + (((size_t)n + 15) & ~(size_t)15);
}

hipError_t launch_resident_sweep(const ResidentArgs &a, bool univariate, hipStream_t s) {
    const size_t lds = resident_lds_bytes(a.n);
    // Raise the dynamic LDS limit of the kernel to what this launch needs (once per size).
    static size_t attr_bytes[2] = {0, 0};
    const void *fn = univariate ? (const void *)k_resident_sweep<true>
                                : (const void *)k_resident_sweep<false>;
    if (lds > attr_bytes[univariate]) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_bytes[univariate] = lds;
    }
    if (univariate)
        hipLaunchKernelGGL((k_resident_sweep<true>), dim3(a.N), dim3(kResidentThreads), lds, s, a);
    else
        hipLaunchKernelGGL((k_resident_sweep<false>), dim3(a.N), dim3(kResidentThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_epilogue(const EpilogueArgs &a, hipStream_t s) {
    const int grid = (a.n + kEpiThreads - 1) / kEpiThreads;
    hipLaunchKernelGGL(k_epilogue, dim3(grid), dim3(kEpiThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace gom
