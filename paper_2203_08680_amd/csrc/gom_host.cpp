// gom_host.cpp -- host side of libgom: instance and linkage-model handling, Welsh-Powell
// colouring, the class-ordered element records, the device arena layout and the generation
// driver behind the C ABI declared in include/gom.h.
#include "../../include/gom.h"
#include "gom_internal.h"
#include "gom_arena.h"

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <map>
#include <new>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

using namespace gom;

// ------------------------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(GOM_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

#define GUARD_BEGIN try {
#define GUARD_END                                                                            \
    }                                                                                        \
    catch (const std::bad_alloc &) {                                                         \
        return fail(GOM_E_NOMEM, "host allocation failed");                                  \
    }                                                                                        \
    catch (...) {                                                                            \
        return fail(GOM_E_ARG, "unexpected internal error");                                 \
    }

// ------------------------------------------------------------------------------------------
// Handles
// ------------------------------------------------------------------------------------------
struct mc_graph {
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int32_t> eu, ev, ew;        // edges as given
    std::vector<int32_t> row_ptr, col, wt;  // CSR, rows ascending by neighbour
    int64_t total_weight = 0;
    int32_t max_degree = 0;
};

struct gom_fos {
    int32_t n_vars = 0;
    int32_t n_sets = 0;
    std::vector<int32_t> ptr, vars;  // each set ascending
    int32_t max_set = 0;
    bool coloured = false;
    int32_t k = 0;
    std::vector<int32_t> colour, class_ptr, class_elems;
};

namespace {

struct Layout {
    size_t st, fit, stripes, E, P, O, rows, cptr, crec, eu, ev, ew, roff, recs, coop, sw, smap,
        split, fdep, fflags, total;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int32_t n, int64_t m, int32_t n_sets, int32_t k, int32_t pop,
                   int64_t rec_words, int64_t n_coop, int64_t sw_words, int64_t n_smap) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    L.st = take(sizeof(DevState));
    L.fit = take(sizeof(int64_t) * GOM_MAX_POP);
    L.stripes = take(sizeof(Stripe) * kStripes);
    L.E = take(sizeof(uint64_t) * (size_t)((n + 63) / 64));
    L.P = take(sizeof(uint64_t) * (size_t)n);
    L.O = take(sizeof(uint64_t) * (size_t)n);
    L.rows = take(sizeof(uint64_t) * (size_t)pop * (size_t)((n + 63) / 64));
    L.cptr = take(sizeof(int32_t) * (size_t)(k + 1));
    L.crec = take(sizeof(int2) * (size_t)k);
    L.eu = take(sizeof(int32_t) * (size_t)m);
    L.ev = take(sizeof(int32_t) * (size_t)m);
    L.ew = take(sizeof(int32_t) * (size_t)m);
    L.roff = take(sizeof(int32_t) * (size_t)(n_sets + 1));
    L.recs = take(sizeof(int32_t) * (size_t)rec_words);
    L.coop = take(sizeof(int32_t) * (size_t)n_coop);
    L.sw = take(sizeof(int32_t) * (size_t)sw_words);
    L.smap = take(sizeof(int4) * (size_t)n_smap);
    L.split = take(n_smap ? kSplitScratchBytes : 0);
    // fused bit-sliced sweep: dependency ranges and chunk flags for up to kFusedMaxGrid chunks
    const bool fused = sw_words > 0 && k <= kFusedMaxClasses;
    L.fdep = take(fused ? sizeof(int4) * (size_t)k * k * kFusedMaxGrid : 0);
    L.fflags = take(fused ? sizeof(uint32_t) * (size_t)k * kFusedMaxGrid : 0);
    L.total = o;
    return L;
}

// Set records in class order, one per class position s, at word offset roff[s] of `words`,
// each on a 16-byte boundary (layout documented in gom_kernels.hip): the set's variables and
// the edges that depend on them, split into outside edges (to a vertex v outside the set) and
// inside edges (both ends in the set, listed once).  16 zero words follow the last record so
// the kernels' fixed-size header reads stay inside the buffer.
struct Records {
    std::vector<int32_t> roff, words;
    std::vector<int2> class_rec;        // per class {first word, stride or 0}
    std::vector<int32_t> class_entries;  // per class: most dependent-edge entries of a record
    std::vector<int32_t> class_members;  // per class: most members of a set
    std::vector<int64_t> class_wsum;     // per class: largest sum of |w| over a set's entries
    std::vector<int64_t> class_wmax;     // per class: largest |w| of an entry
};

constexpr int kSmallSet = 14;         // members held in a small record's header
constexpr int kSmallPosShift = 27;    // bits 27..30 of a small entry: member position
constexpr int32_t kMaxVertexSmall = 1 << kSmallPosShift;  // vertex limit of a state

// Class positions of the sets swept by a whole block (general FOS only), per class in two
// groups: sets of up to kCoopSmallBlock members (256-thread blocks), then larger ones
// (1024-thread blocks).  Group g of class c: pos[ptr[2c + g] .. ptr[2c + g + 1]); the
// largest set of each group in max_members[2c + g].  A class with fewer than kSplitBelow
// large sets in its two groups together takes the split sweep for all of them instead
// (split[c] set): its blocks, one per chunk of kSplitMembers members, are
// smap[smap_ptr[c] .. smap_ptr[c + 1]) = {slot (the set's index among the class's large
// sets), class position, first member, 0}.
struct CoopSets {
    std::vector<int32_t> ptr, pos, max_members, smap_ptr;
    std::vector<uint8_t> split;
    std::vector<int4> smap;
};

CoopSets coop_sets(const gom_fos &f, bool univariate) {
    CoopSets C;
    C.ptr.assign(2 * (size_t)f.k + 1, 0);
    C.max_members.assign(2 * (size_t)f.k, 0);
    C.smap_ptr.assign((size_t)f.k + 1, 0);
    C.split.assign((size_t)f.k, 0);
    for (int32_t c = 0; c < f.k; ++c) {
        for (int grp = 0; grp < 2; ++grp) {
            const size_t q = 2 * (size_t)c + grp;
            if (!univariate)
                for (int32_t t = f.class_ptr[c]; t < f.class_ptr[(size_t)c + 1]; ++t) {
                    const int32_t j = f.class_elems[t];
                    const int32_t nm = f.ptr[(size_t)j + 1] - f.ptr[j];
                    if (nm < kCoopMinMembers || nm > kCoopMaxMembers) continue;
                    if ((nm > kCoopSmallBlock) != (grp == 1)) continue;
                    C.pos.push_back(t - f.class_ptr[c]);
                    C.max_members[q] = std::max(C.max_members[q], nm);
                }
            C.ptr[q + 1] = (int32_t)C.pos.size();
        }
        const int32_t first = C.ptr[2 * (size_t)c], n_large = C.ptr[2 * (size_t)c + 2] - first;
        if (n_large > 0 && n_large < kSplitBelow) {
            C.split[c] = 1;
            for (int32_t slot = 0; slot < n_large; ++slot) {
                const int32_t p = C.pos[(size_t)first + slot];
                const int32_t j = f.class_elems[(size_t)f.class_ptr[c] + p];
                const int32_t nm = f.ptr[(size_t)j + 1] - f.ptr[j];
                for (int32_t k0 = 0; k0 < nm; k0 += kSplitMembers)
                    C.smap.push_back(make_int4(slot, p, k0, 0));
            }
        }
        C.smap_ptr[(size_t)c + 1] = (int32_t)C.smap.size();
    }
    return C;
}

// Truth tables of a univariate set {u} with at most 4 edges, for the bit-sliced sweep: bit p
// of the low half = (flip gain > 0), of the high half = (gain == 0), for the pattern p of
// edges whose far end carries the same gene (bit e set: edge e gains +w_e).  Edges beyond the
// vertex's degree have weight 0.
uint32_t uni_tables(const mc_graph &g, int32_t u) {
    const int32_t nd = g.row_ptr[(size_t)u + 1] - g.row_ptr[u];
    if (nd > 4) return 0;
    int64_t wl[4] = {0, 0, 0, 0}, tot = 0;
    for (int32_t e = 0; e < nd; ++e) {
        wl[e] = g.wt[(size_t)g.row_ptr[u] + e];
        tot += wl[e];
    }
    uint32_t tables = 0;
    for (uint32_t pt = 0; pt < 16; ++pt) {
        int64_t d = -tot;
        for (int e = 0; e < 4; ++e)
            if (pt >> e & 1u) d += 2 * wl[e];
        tables |= (uint32_t)(d > 0) << pt | (uint32_t)(d == 0) << (pt + 16);
    }
    return tables;
}

// The bit-sliced schedule handles univariate FOS on graphs of degree <= 4 whose per-vertex
// sums of |w| stay below 2^30 (its per-solution gains are int32).
// max_abs_out (may be null): the largest sum of |w| over a vertex's edges, a bound on the
// size of one flip's fitness change.
bool swar_eligible(const mc_graph &g, const gom_fos &f, int64_t *max_abs_out = nullptr) {
    if (f.max_set != 1 || g.max_degree > 4) return false;
    int64_t max_abs = 0;
    for (int32_t v = 0; v < g.n; ++v) {
        int64_t t = 0;
        for (int32_t r = g.row_ptr[v]; r < g.row_ptr[(size_t)v + 1]; ++r)
            t += g.wt[r] < 0 ? -(int64_t)g.wt[r] : (int64_t)g.wt[r];
        max_abs = std::max(max_abs, t);
    }
    if (max_abs_out) *max_abs_out = max_abs;
    return max_abs < ((int64_t)1 << 30);
}

int32_t swar_stride(int32_t n_sets) { return (n_sets + 63) & ~63; }

// The bit-sliced sweep's table (kSwRows arrays of swar_stride words, entry s = class position
// s of the colour classes in order): u, its truth tables, its neighbours (u itself where the
// vertex has fewer than 4), their weights (0 there).
std::vector<int32_t> build_swar(const mc_graph &g, const gom_fos &f) {
    const size_t ss = (size_t)swar_stride(f.n_sets);
    std::vector<int32_t> T(kSwRows * ss, 0);
    int32_t s = 0;
    for (int32_t c = 0; c < f.k; ++c)
        for (int32_t t = f.class_ptr[c]; t < f.class_ptr[(size_t)c + 1]; ++t, ++s) {
            const int32_t u = f.vars[f.ptr[f.class_elems[t]]];
            T[kSwU * ss + s] = u;
            T[kSwTables * ss + s] = (int32_t)uni_tables(g, u);
            const int32_t r0 = g.row_ptr[u], nd = g.row_ptr[(size_t)u + 1] - r0;
            for (int e = 0; e < 4; ++e) {
                T[(kSwV + e) * ss + s] = e < nd ? g.col[(size_t)r0 + e] : u;
                T[(kSwW + e) * ss + s] = e < nd ? g.wt[(size_t)r0 + e] : 0;
            }
        }
    return T;
}

// Chunks of the fused bit-sliced sweep: class c's positions cut into `grid` chunks of
// clen[c] = ceil(|class| / grid) positions.  dep[(c * grid + x) * k + c2] holds the chunks of
// class c2 with a set whose variable is a variable of chunk x of class c or a neighbour of one
// (the chunks that write what chunk x reads, or read what it writes) as two ranges {lo0, hi0,
// lo1, hi1}: the sorted chunk ids split at their widest gap, so that the wrap-around edges of
// a torus cost two short ranges instead of one that spans the class; an unused range is
// {0, -1}.  Returns false when the two ranges of some entry span more than kFusedMaxDepChunks
// chunks together.
bool fused_deps(const mc_graph &g, const gom_fos &f, int grid, std::vector<int32_t> &clen,
                std::vector<int4> &dep) {
    const int k = f.k;
    const size_t n = (size_t)g.n;
    clen.assign((size_t)k, 1);
    for (int c = 0; c < k; ++c) {
        const int32_t cs = f.class_ptr[(size_t)c + 1] - f.class_ptr[c];
        clen[(size_t)c] = std::max<int32_t>(1, (cs + grid - 1) / grid);
    }
    std::vector<int32_t> at((size_t)k * n, -1);  // chunk of class c holding variable v
    for (int c = 0; c < k; ++c)
        for (int32_t t = f.class_ptr[c]; t < f.class_ptr[(size_t)c + 1]; ++t) {
            const int32_t u = f.vars[f.ptr[f.class_elems[t]]];
            at[(size_t)c * n + u] = (t - f.class_ptr[c]) / clen[(size_t)c];
        }
    dep.assign((size_t)k * grid * k, make_int4(0, -1, 0, -1));
    std::vector<int32_t> ids;
    for (int c = 0; c < k; ++c) {
        const int32_t c0 = f.class_ptr[c], cs = f.class_ptr[(size_t)c + 1] - c0;
        for (int32_t x = 0; x < grid; ++x) {
            const int32_t p0 = x * clen[(size_t)c], p1 = std::min(p0 + clen[(size_t)c], cs);
            for (int c2 = 0; c2 < k; ++c2) {
                if (c2 == c) continue;
                ids.clear();
                for (int32_t p = p0; p < p1; ++p) {
                    const int32_t u = f.vars[f.ptr[f.class_elems[c0 + p]]];
                    auto add = [&](int32_t w) {
                        const int32_t y = at[(size_t)c2 * n + w];
                        if (y >= 0) ids.push_back(y);
                    };
                    add(u);
                    for (int32_t q = g.row_ptr[u]; q < g.row_ptr[(size_t)u + 1]; ++q)
                        add(g.col[q]);
                }
                if (ids.empty()) continue;
                std::sort(ids.begin(), ids.end());
                ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
                size_t cut = ids.size() - 1;  // split after ids[cut] at the widest gap
                int32_t gap = 0;
                for (size_t q = 0; q + 1 < ids.size(); ++q)
                    if (ids[q + 1] - ids[q] > gap) {
                        gap = ids[q + 1] - ids[q];
                        cut = q;
                    }
                int4 &r = dep[((size_t)c * grid + x) * k + c2];
                r = make_int4(ids.front(), ids[cut], 0, -1);
                if (cut + 1 < ids.size()) {
                    r.z = ids[cut + 1];
                    r.w = ids.back();
                }
                const int32_t span = (r.y - r.x + 1) + (r.w >= r.z ? r.w - r.z + 1 : 0);
                if (span > kFusedMaxDepChunks) return false;
            }
        }
    }
    return true;
}

int build_records(const mc_graph &g, const gom_fos &f, bool univariate, Records &R) {
    const int32_t S = f.n_sets;
    std::vector<int32_t> pos((size_t)g.n, -1), owner((size_t)g.n, -1);
    R.roff.assign((size_t)S + 1, 0);
    R.words.clear();
    auto pad4 = [&]() {
        while (R.words.size() & 3) R.words.push_back(0);
    };
    std::vector<std::pair<int32_t, int32_t>> ent;  // (x, w)
    std::vector<int32_t> ends;
    R.class_rec.assign((size_t)f.k, make_int2(0, 0));
    R.class_entries.assign((size_t)f.k, 0);
    R.class_members.assign((size_t)f.k, 1);
    R.class_wsum.assign((size_t)f.k, 0);
    R.class_wmax.assign((size_t)f.k, 0);
    int32_t s = 0;
    for (int32_t c = 0; c < f.k; ++c) {
        const size_t class_first = R.words.size();
        const int32_t s_first = s;
        for (int32_t t = f.class_ptr[c]; t < f.class_ptr[(size_t)c + 1]; ++t, ++s) {
            if (R.words.size() >= (size_t)INT32_MAX / 2)
                return fail(GOM_E_RANGE, "set records exceed 2^30 words");
            R.roff[s] = (int32_t)R.words.size();
            const int32_t j = f.class_elems[t];
            const int32_t b = f.ptr[j], e = f.ptr[(size_t)j + 1], nm = e - b;
            if (univariate) {
                const int32_t u = f.vars[b];
                const int32_t nd = g.row_ptr[(size_t)u + 1] - g.row_ptr[u];
                R.class_entries[c] = std::max(R.class_entries[c], nd);
                R.words.insert(R.words.end(), {u, nd, 0, 0});
                for (int32_t r = g.row_ptr[u]; r < g.row_ptr[(size_t)u + 1]; ++r) {
                    R.words.push_back(g.col[r]);
                    R.words.push_back(g.wt[r]);
                }
                pad4();
                continue;
            }
            for (int32_t q = b; q < e; ++q) {
                owner[f.vars[q]] = j;
                pos[f.vars[q]] = q - b;
            }
            const bool small = nm <= kSmallSet;
            ent.clear();
            ends.clear();
            for (int32_t q = 0; q < nm; ++q) {
                const int32_t u = f.vars[b + q];
                for (int32_t r = g.row_ptr[u]; r < g.row_ptr[(size_t)u + 1]; ++r) {
                    const int32_t v = g.col[r];
                    if (owner[v] == j) {
                        if (pos[v] > q)
                            ent.push_back({small ? (int32_t)(0x80000000u |
                                                             ((uint32_t)q << kSmallPosShift) |
                                                             (uint32_t)pos[v])
                                                 : ~pos[v],
                                           g.wt[r]});
                    } else {
                        ent.push_back({small ? (int32_t)(((uint32_t)q << kSmallPosShift) |
                                                         (uint32_t)v)
                                             : v,
                                       g.wt[r]});
                    }
                }
                ends.push_back((int32_t)ent.size());
            }
            const int32_t nd = (int32_t)ent.size();
            R.class_entries[c] = std::max(R.class_entries[c], nd);
            R.class_members[c] = std::max(R.class_members[c], nm);
            int64_t wsum = 0;
            for (const auto &xw : ent) {
                const int64_t aw = std::llabs((long long)xw.second);
                wsum += aw;
                R.class_wmax[c] = std::max(R.class_wmax[c], aw);
            }
            R.class_wsum[c] = std::max(R.class_wsum[c], wsum);
            R.words.push_back(nm);
            R.words.push_back(nd);
            if (small) {
                for (int32_t q = 0; q < kSmallSet; ++q) R.words.push_back(q < nm ? f.vars[b + q] : -1);
            } else {
                for (int q = 0; q < 14; ++q) R.words.push_back(0);
                for (int32_t q = 0; q < nm; ++q) R.words.push_back(f.vars[b + q]);
                for (int32_t q = 0; q < nm; ++q) R.words.push_back(ends[q]);
                pad4();
            }
            for (const auto &xw : ent) {
                R.words.push_back(xw.first);
                R.words.push_back(xw.second);
            }
            pad4();
        }
        // Pad the class's records to one size when that costs at most a quarter more words:
        // the kernels then locate record p at first + p * stride without reading roff.
        const int32_t cnt = s - s_first;
        if (cnt == 0) continue;
        int32_t longest = 0;
        for (int32_t q = s_first; q < s; ++q) {
            const int32_t len =
                (q + 1 < s ? R.roff[q + 1] : (int32_t)R.words.size()) - R.roff[q];
            longest = std::max(longest, len);
        }
        const size_t used = R.words.size() - class_first;
        if ((size_t)longest * (size_t)cnt * 4 <= used * 5) {
            std::vector<int32_t> block(R.words.begin() + (ptrdiff_t)class_first, R.words.end());
            R.words.resize(class_first);
            for (int32_t q = s_first; q < s; ++q) {
                const size_t b0 = (size_t)R.roff[q] - class_first;
                const size_t b1 = (q + 1 < s ? (size_t)R.roff[q + 1] - class_first : block.size());
                R.roff[q] = (int32_t)R.words.size();
                R.words.insert(R.words.end(), block.begin() + (ptrdiff_t)b0,
                               block.begin() + (ptrdiff_t)b1);
                R.words.resize(R.words.size() + (size_t)longest - (b1 - b0), 0);
            }
            R.class_rec[c] = make_int2((int32_t)class_first, longest);
        } else {
            R.class_rec[c] = make_int2((int32_t)class_first, 0);
        }
    }
    R.roff[S] = (int32_t)R.words.size();
    // zero tail: the kernels fetch the first entry batches of a record together with its
    // header (up to 48 words past the end of the last record), the batched class launches a
    // record's first kRecordTailWords words
    for (int q = 0; q < kRecordTailWords; ++q) R.words.push_back(0);
    return GOM_OK;
}

}  // namespace

// Default least class size (sets) for the general bit-sliced sweep: with one set per lane a
// smaller class leaves too few waves. A 3-regular graph's classes of about 10^4
// neighbourhoods are swept faster by the class sweep, the 10^6-vertex torus's of 1.25*10^5
// neighbourhoods 2.6 times slower.
constexpr int32_t kGsMinSets = 32768;

// Largest instance (vertices) GOM_SCHED_AUTO gives the resident schedule. Its N blocks (one a
// solution) occupy N compute units, so past about a thousand vertices the class launches,
// which spread each class over the whole device, are faster. Per generation, resident against
// class launch (tori with neighbourhoods, N = 64): 45.9 / 47.4 us at 32x32, 53.0 / 47.9 at
// 48x48, 55.3 / 47.4 at 64x64, 80.0 / 56.7 at 100x100; 740 / 192 us on a 10^5-vertex
// 3-regular graph with neighbourhoods, N = 32.
constexpr int32_t kResidentAutoMaxVertices = 1536;

struct gom_state {
    int static_dev = -1;                // device whose static arena holds the state, or -1
    bool h_st_pinned = true;            // h_st from hipHostMalloc (else new[])
    bool fused_ok = false;              // the fused bit-sliced sweep can run this state
    bool fused_use = false;             // ... and is used for whole generations
    bool fused_narrow = false;          // its per-block fitness sums fit in int32
    int fused_grid = 0;
    std::vector<int32_t> fused_clen;    // chunk length per class
    uint32_t fused_epoch = 0;           // stamp of the last fused launch
    int4 *d_fdep = nullptr;
    uint32_t *d_fflags = nullptr;
    int32_t n = 0, N = 0, n_sets = 0, k = 0, max_class = 0;
    int64_t m = 0;
    uint64_t seed = 0;
    int rule = 0, order = 0;
    bool univariate = false;
    int32_t max_set = 0;                // largest set of the FOS
    std::vector<int32_t> class_ptr;
    char *arena = nullptr;
    Layout L{};
    DevState *d_st = nullptr;
    int64_t *d_fit = nullptr;
    Stripe *d_stripes = nullptr;
    uint64_t *d_E = nullptr, *d_P = nullptr, *d_O = nullptr, *d_rows = nullptr;
    int32_t *d_cptr = nullptr;
    int sched = GOM_SCHED_CLASS_LAUNCH;  // schedule in use
    bool resident_ok = false;            // resident schedule fits instance and device
    bool resident_plds = false;          // ... with a copy of P in LDS as well
    size_t lds_max = 0;                  // LDS bytes a block may use on the device
    bool bitsliced_ok = false;           // bit-sliced schedule fits the instance
    bool swar_narrow = false;            // its per-block fitness sums fit in int32
    bool partition = false;              // every variable in exactly one set
    bool fi = false;                     // forced improvement after each generation's classes
    int32_t *d_eu = nullptr, *d_ev = nullptr, *d_ew = nullptr;
    int32_t *d_roff = nullptr, *d_recs = nullptr;
    int2 *d_crec = nullptr;
    std::vector<int2> class_rec;  // host copy of the per-class record placement
    std::vector<int32_t> class_entries;  // per class: most entries of one of its records
    std::vector<int32_t> class_members;  // per class: most members of one of its sets
    std::vector<int8_t> gs_wbits;        // per class: bits of its largest |w| when the general
                                         // bit-sliced sweep takes it, else 0
    std::vector<int64_t> class_wsum, class_wmax;  // per class (see Records)
    int32_t gs_min_sets = kGsMinSets;    // smallest class the general bit-sliced sweep takes
    bool swar_uni = false;               // the univariate bit-sliced sweep fits the instance
    bool staged_use = false;            // per-class sweeps of small general sets staged
    std::vector<int32_t> coop_ptr, coop_max;  // large sets per class (block-cooperative)
    int32_t *d_coop = nullptr;                // their class positions
    int32_t *d_sw = nullptr;                  // bit-sliced sweep table (when eligible)
    int32_t sw_stride = 0;
    std::vector<uint8_t> split;               // per class: split sweep (few large sets)
    std::vector<int32_t> smap_ptr;            // ... its blocks in d_smap
    int4 *d_smap = nullptr;
    uint64_t *d_split_D = nullptr;            // split sweep scratch (per slot)
    int64_t *d_split_delta = nullptr;
    int32_t *d_split_sel = nullptr;
    int32_t g_host = 0;                 // next generation index to enqueue
    int32_t open_next = -1;             // class position where an open generation resumes
    int32_t g_base = 0;                 // generation at which attempted_base was set
    int64_t attempted_base = 0;
    DevState *h_st = nullptr;           // two pinned host slots
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    int max_grid = 2048;                // grid cap of the class sweeps
    int64_t swar_abs = 0;               // largest per-vertex |weight| sum (bit-sliced sweep)
    int sweep_threads = 256;            // class-launch block size (64..512)
    int timing = 0;                     // sample period of the sweep-launch events (0 = off)
    int64_t sweep_launches = 0;         // sweep launches enqueued (for the sampling)
    std::vector<hipEvent_t> tev;        // begin/end pairs
    size_t tev_used = 0;
    double t_ms = 0.0;
    int64_t t_launches = 0;
};

// ------------------------------------------------------------------------------------------
// Graph
// ------------------------------------------------------------------------------------------
extern "C" const char *gom_last_error(void) { return g_err.c_str(); }
extern "C" int gom_version(void) { return 2; }

extern "C" int mc_graph_load(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                             const int32_t *w, mc_graph **out) {
    GUARD_BEGIN
    if (!u || !v || !out) return fail(GOM_E_ARG, "mc_graph_load: null argument");
    if (n < 1) return fail(GOM_E_RANGE, "mc_graph_load: n_vertices must be >= 1 (got %d)", n);
    if (m < 1 || 2 * m >= ((int64_t)1 << 31))
        return fail(GOM_E_RANGE, "mc_graph_load: n_edges must be in [1, 2^30) (got %lld)",
                    (long long)m);
    for (int64_t e = 0; e < m; ++e) {
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n)
            return fail(GOM_E_GRAPH, "mc_graph_load: edge %lld endpoint out of range",
                        (long long)e);
        if (u[e] == v[e])
            return fail(GOM_E_GRAPH, "mc_graph_load: edge %lld is a self-loop", (long long)e);
        // a step negates the weight of an edge it uncuts, so -w must be an int32 too
        if (w && w[e] == INT32_MIN)
            return fail(GOM_E_RANGE, "mc_graph_load: edge %lld has weight -2^31 (|w| must be "
                        "below 2^31)", (long long)e);
    }
    auto *g = new mc_graph;
    g->n = n;
    g->m = m;
    g->eu.assign(u, u + m);
    g->ev.assign(v, v + m);
    if (w) g->ew.assign(w, w + m);
    else g->ew.assign((size_t)m, 1);
    g->row_ptr.assign((size_t)n + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        g->row_ptr[(size_t)u[e] + 1]++;
        g->row_ptr[(size_t)v[e] + 1]++;
    }
    for (int32_t x = 0; x < n; ++x) g->row_ptr[(size_t)x + 1] += g->row_ptr[x];
    std::vector<int32_t> fill(g->row_ptr.begin(), g->row_ptr.end() - 1);
    std::vector<std::pair<int32_t, int32_t>> adj((size_t)(2 * m));
    for (int64_t e = 0; e < m; ++e) {
        adj[(size_t)fill[u[e]]++] = {v[e], g->ew[e]};
        adj[(size_t)fill[v[e]]++] = {u[e], g->ew[e]};
        g->total_weight += g->ew[e];
    }
    g->col.resize((size_t)(2 * m));
    g->wt.resize((size_t)(2 * m));
    for (int32_t x = 0; x < n; ++x) {
        auto b = adj.begin() + g->row_ptr[x], e = adj.begin() + g->row_ptr[(size_t)x + 1];
        std::sort(b, e);
        for (auto it = b; it != e; ++it) {
            if (it != b && it->first == (it - 1)->first) {
                const int32_t y = it->first;
                delete g;
                return fail(GOM_E_GRAPH, "mc_graph_load: edge {%d, %d} appears twice", x, y);
            }
            g->col[(size_t)(it - adj.begin())] = it->first;
            g->wt[(size_t)(it - adj.begin())] = it->second;
        }
        g->max_degree = std::max(g->max_degree, (int32_t)(e - b));
    }
    *out = g;
    return GOM_OK;
    GUARD_END
}

extern "C" int mc_graph_info(const mc_graph *g, int32_t *n, int64_t *m, int64_t *total_weight,
                             int32_t *max_degree) {
    if (!g) return fail(GOM_E_ARG, "mc_graph_info: null graph");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (total_weight) *total_weight = g->total_weight;
    if (max_degree) *max_degree = g->max_degree;
    return GOM_OK;
}

extern "C" int mc_graph_csr(const mc_graph *g, int32_t *row_ptr, int32_t *col, int32_t *w) {
    if (!g || !row_ptr || !col || !w) return fail(GOM_E_ARG, "mc_graph_csr: null argument");
    std::copy(g->row_ptr.begin(), g->row_ptr.end(), row_ptr);
    std::copy(g->col.begin(), g->col.end(), col);
    std::copy(g->wt.begin(), g->wt.end(), w);
    return GOM_OK;
}

extern "C" void mc_graph_free(mc_graph *g) { delete g; }

// ------------------------------------------------------------------------------------------
// FOS
// ------------------------------------------------------------------------------------------
extern "C" int gom_fos_build(const mc_graph *g, int kind, gom_fos **out) {
    GUARD_BEGIN
    if (!g || !out) return fail(GOM_E_ARG, "gom_fos_build: null argument");
    if (kind != GOM_FOS_UNIVARIATE && kind != GOM_FOS_NEIGHBOURHOOD)
        return fail(GOM_E_ARG, "gom_fos_build: unknown kind %d", kind);
    auto *f = new gom_fos;
    f->n_vars = g->n;
    f->n_sets = g->n;
    f->ptr.assign((size_t)g->n + 1, 0);
    for (int32_t v = 0; v < g->n; ++v) {
        if (kind == GOM_FOS_UNIVARIATE) {
            f->vars.push_back(v);
        } else {
            // {v} + N(v), ascending: the CSR row is already ascending; insert v in place.
            const int32_t b = g->row_ptr[v], e = g->row_ptr[(size_t)v + 1];
            bool put = false;
            for (int32_t q = b; q < e; ++q) {
                if (!put && g->col[q] > v) { f->vars.push_back(v); put = true; }
                f->vars.push_back(g->col[q]);
            }
            if (!put) f->vars.push_back(v);
        }
        f->ptr[(size_t)v + 1] = (int32_t)f->vars.size();
        f->max_set = std::max(f->max_set, f->ptr[(size_t)v + 1] - f->ptr[v]);
    }
    *out = f;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_fos_from_sets(const mc_graph *g, int32_t n_sets, const int32_t *ptr,
                                 const int32_t *vars, gom_fos **out) {
    GUARD_BEGIN
    if (!g || !ptr || !vars || !out) return fail(GOM_E_ARG, "gom_fos_from_sets: null argument");
    if (n_sets < 1) return fail(GOM_E_ARG, "gom_fos_from_sets: n_sets must be >= 1");
    if (ptr[0] != 0) return fail(GOM_E_ARG, "gom_fos_from_sets: ptr[0] must be 0");
    std::vector<int32_t> seen((size_t)g->n, -1);
    std::vector<char> covered((size_t)g->n, 0);
    auto *f = new gom_fos;
    f->n_vars = g->n;
    f->n_sets = n_sets;
    f->ptr.assign(ptr, ptr + n_sets + 1);
    for (int32_t j = 0; j < n_sets; ++j) {
        if (ptr[j + 1] <= ptr[j]) {
            delete f;
            return fail(GOM_E_ARG, "gom_fos_from_sets: set %d is empty or ptr decreases", j);
        }
        std::vector<int32_t> s(vars + ptr[j], vars + ptr[j + 1]);
        for (int32_t x : s) {
            if (x < 0 || x >= g->n) {
                delete f;
                return fail(GOM_E_ARG, "gom_fos_from_sets: variable %d out of range in set %d",
                            x, j);
            }
            if (seen[x] == j) {
                delete f;
                return fail(GOM_E_ARG, "gom_fos_from_sets: variable %d twice in set %d", x, j);
            }
            seen[x] = j;
            covered[x] = 1;
        }
        std::sort(s.begin(), s.end());
        f->vars.insert(f->vars.end(), s.begin(), s.end());
        f->max_set = std::max(f->max_set, (int32_t)s.size());
    }
    for (int32_t x = 0; x < g->n; ++x)
        if (!covered[x]) {
            delete f;
            return fail(GOM_E_ARG, "gom_fos_from_sets: variable %d is in no set (FOS must be "
                                   "complete)", x);
        }
    *out = f;
    return GOM_OK;
    GUARD_END
}

// ------------------------------------------------------------------------------------------
// Fixed linkage tree (Section 4.1): UPGMA over the variables, with the absolute edge weight as
// the similarity of two variables (0 when they share no edge).  Clusters are merged pair by
// pair, always a pair with the largest average similarity between their members; ties go to
// the smaller combined size, then to the lower cluster ids (variables are clusters 0..n-1,
// merged clusters get n, n+1, ... in creation order).  With a bound, only pairs whose union
// has at most `bound` members may merge, and the tree stops when no such pair is left.  The
// set of all variables is not part of the tree.
//
// Two clusters that share no edge have average similarity 0, and every pair that shares one
// has a positive average, so the merges run in two phases: first the pairs with a positive
// average, from a heap of candidate pairs (a pair's summed similarity never changes while
// both are unmerged, so stale entries are only those of merged clusters); then, when no
// allowed positive pair is left, pairs of average 0, for which the tie rule picks the two
// smallest clusters by (size, id).
// ------------------------------------------------------------------------------------------
namespace {

struct LtCand {
    int64_t W;    // summed similarity between the two clusters
    int64_t sz;   // size product
    int32_t sum;  // size sum
    int32_t lo, hi;
};

// a ranks below b: smaller average, then larger size sum, then larger ids
struct LtLess {
    bool operator()(const LtCand &a, const LtCand &b) const {
        const __int128 x = (__int128)a.W * b.sz, y = (__int128)b.W * a.sz;
        if (x != y) return x < y;
        if (a.sum != b.sum) return a.sum > b.sum;
        if (a.lo != b.lo) return a.lo > b.lo;
        return a.hi > b.hi;
    }
};

}  // namespace

extern "C" int gom_fos_build_lt(const mc_graph *g, int32_t bound, gom_fos **out) {
    GUARD_BEGIN
    if (!g || !out) return fail(GOM_E_ARG, "gom_fos_build_lt: null argument");
    if (bound < 0 || bound == 1) return fail(GOM_E_ARG, "gom_fos_build_lt: bound must be 0 or >= 2");
    const int32_t n = g->n;
    const int64_t cap = bound ? bound : (int64_t)n;  // largest allowed set
    std::vector<int32_t> size((size_t)n), parent_a, parent_b;
    std::vector<char> alive((size_t)n, 1);
    std::vector<std::unordered_map<int32_t, int64_t>> W((size_t)n);
    for (int32_t v = 0; v < n; ++v) {
        size[v] = 1;
        for (int32_t r = g->row_ptr[v]; r < g->row_ptr[(size_t)v + 1]; ++r) {
            const int64_t w = g->wt[r] < 0 ? -(int64_t)g->wt[r] : (int64_t)g->wt[r];
            if (w) W[v][g->col[r]] += w;
        }
    }
    std::priority_queue<LtCand, std::vector<LtCand>, LtLess> heap;
    auto push = [&](int32_t a, int32_t b, int64_t w) {
        const int64_t sum = (int64_t)size[a] + size[b];
        if (w <= 0 || sum > cap) return;
        heap.push({w, (int64_t)size[a] * size[b], (int32_t)sum, std::min(a, b), std::max(a, b)});
    };
    for (int32_t v = 0; v < n; ++v)
        for (const auto &kv : W[v])
            if (kv.first > v) push(v, kv.first, kv.second);
    int32_t n_alive = n;
    auto merge = [&](int32_t a, int32_t b) {
        const int32_t c = (int32_t)size.size();
        size.push_back(size[a] + size[b]);
        alive.push_back(1);
        alive[a] = alive[b] = 0;
        parent_a.push_back(a);
        parent_b.push_back(b);
        W.emplace_back();
        std::unordered_map<int32_t, int64_t> &wc = W.back();
        for (int32_t x : {a, b}) {
            for (const auto &kv : W[x])
                if (alive[kv.first]) wc[kv.first] += kv.second;
            std::unordered_map<int32_t, int64_t>().swap(W[x]);
        }
        for (const auto &kv : wc) {
            W[kv.first].erase(a);
            W[kv.first].erase(b);
            W[kv.first][c] = kv.second;
            push(c, kv.first, kv.second);
        }
        --n_alive;
    };
    // the merge that would join every variable is never made
    auto root = [&](int32_t a, int32_t b) { return (int64_t)size[a] + size[b] >= n; };
    bool stop = false;
    while (!heap.empty() && n_alive > 1) {
        const LtCand t = heap.top();
        heap.pop();
        if (!alive[t.lo] || !alive[t.hi]) continue;
        if (root(t.lo, t.hi)) {
            stop = true;
            break;
        }
        merge(t.lo, t.hi);
    }
    if (!stop && n_alive > 1) {
        // average 0 for every remaining allowed pair: two smallest clusters by (size, id)
        using SI = std::pair<int32_t, int32_t>;
        std::priority_queue<SI, std::vector<SI>, std::greater<SI>> small;
        for (int32_t c = 0; c < (int32_t)size.size(); ++c)
            if (alive[c]) small.push({size[c], c});
        while (small.size() >= 2) {
            const SI x = small.top();
            small.pop();
            const SI y = small.top();
            if ((int64_t)x.first + y.first > cap || root(x.second, y.second)) break;
            small.pop();
            merge(std::min(x.second, y.second), std::max(x.second, y.second));
            small.push({size.back(), (int32_t)size.size() - 1});
        }
    }
    // sets: the variables, then the merged clusters in creation order (members ascending)
    auto *f = new gom_fos;
    f->n_vars = n;
    const int32_t total = (int32_t)size.size();
    f->n_sets = total;
    f->ptr.assign((size_t)total + 1, 0);
    std::vector<int32_t> first((size_t)total), len((size_t)total);
    for (int32_t v = 0; v < n; ++v) {
        f->vars.push_back(v);
        f->ptr[(size_t)v + 1] = v + 1;
    }
    for (int32_t c = n; c < total; ++c) {
        std::vector<int32_t> mem;
        for (int32_t part : {parent_a[(size_t)(c - n)], parent_b[(size_t)(c - n)]})
            mem.insert(mem.end(), f->vars.begin() + f->ptr[part], f->vars.begin() + f->ptr[(size_t)part + 1]);
        std::sort(mem.begin(), mem.end());
        f->vars.insert(f->vars.end(), mem.begin(), mem.end());
        f->ptr[(size_t)c + 1] = (int32_t)f->vars.size();
        f->max_set = std::max(f->max_set, (int32_t)mem.size());
    }
    f->max_set = std::max(f->max_set, (int32_t)1);
    *out = f;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_fos_info(const gom_fos *f, int32_t *n_sets, int64_t *n_members,
                            int32_t *max_set) {
    if (!f) return fail(GOM_E_ARG, "gom_fos_info: null fos");
    if (n_sets) *n_sets = f->n_sets;
    if (n_members) *n_members = (int64_t)f->vars.size();
    if (max_set) *max_set = f->max_set;
    return GOM_OK;
}

extern "C" int gom_fos_get(const gom_fos *f, int32_t *ptr, int32_t *vars) {
    if (!f || !ptr || !vars) return fail(GOM_E_ARG, "gom_fos_get: null argument");
    std::copy(f->ptr.begin(), f->ptr.end(), ptr);
    std::copy(f->vars.begin(), f->vars.end(), vars);
    return GOM_OK;
}

extern "C" void gom_fos_free(gom_fos *f) { delete f; }

// ------------------------------------------------------------------------------------------
// Colouring: first-fit in Welsh-Powell order (decreasing LMIG degree, then increasing index).
// The LMIG neighbours of set j are the sets containing a variable of N[F_j] (F_j and the
// graph neighbours of its members); they are enumerated through a variable -> sets index
// with a stamp array, so the LMIG is never stored.  First-fit over this order gives exactly
// the classes of the colour-by-colour Welsh-Powell sweep.
// ------------------------------------------------------------------------------------------
extern "C" int gom_colour(const mc_graph *g, gom_fos *f, int32_t *n_colours) {
    GUARD_BEGIN
    if (!g || !f) return fail(GOM_E_ARG, "gom_colour: null argument");
    if (f->n_vars != g->n) return fail(GOM_E_ARG, "gom_colour: FOS built for another graph");
    const int32_t S = f->n_sets;
    std::vector<int32_t> vs_ptr((size_t)g->n + 1, 0), vs(f->vars.size());
    for (int32_t x : f->vars) vs_ptr[(size_t)x + 1]++;
    for (int32_t x = 0; x < g->n; ++x) vs_ptr[(size_t)x + 1] += vs_ptr[x];
    {
        std::vector<int32_t> fill(vs_ptr.begin(), vs_ptr.end() - 1);
        for (int32_t j = 0; j < S; ++j)
            for (int32_t t = f->ptr[j]; t < f->ptr[(size_t)j + 1]; ++t)
                vs[(size_t)fill[f->vars[t]]++] = j;
    }
    auto for_conflicts = [&](int32_t j, auto &&fn) {
        for (int32_t t = f->ptr[j]; t < f->ptr[(size_t)j + 1]; ++t) {
            const int32_t u = f->vars[t];
            for (int32_t a = vs_ptr[u]; a < vs_ptr[(size_t)u + 1]; ++a) fn(vs[a]);
            for (int32_t q = g->row_ptr[u]; q < g->row_ptr[(size_t)u + 1]; ++q) {
                const int32_t x = g->col[q];
                for (int32_t a = vs_ptr[x]; a < vs_ptr[(size_t)x + 1]; ++a) fn(vs[a]);
            }
        }
    };
    // LMIG degrees: each set's distinct conflicting sets, counted with a stamp array.  The
    // sets are split into contiguous ranges over host threads, each with its own stamps; the
    // degrees do not depend on the split.
    std::vector<int64_t> deg((size_t)S, 0);
    auto degrees = [&](int32_t j0, int32_t j1) {
        std::vector<int32_t> stamp((size_t)S, -1);
        for (int32_t j = j0; j < j1; ++j) {
            int64_t d = 0;
            stamp[j] = j;
            for_conflicts(j, [&](int32_t k) {
                if (stamp[k] != j) { stamp[k] = j; ++d; }
            });
            deg[j] = d;
        }
    };
    const int64_t visits = (int64_t)f->vars.size() * (1 + g->max_degree);
    const int nth = (int)std::min<int64_t>(
        std::max(1u, std::min(16u, std::thread::hardware_concurrency())),
        std::max<int64_t>(1, visits / (1 << 20)));
    if (nth <= 1) {
        degrees(0, S);
    } else {
        std::vector<std::thread> pool;
        for (int q = 0; q < nth; ++q)
            pool.emplace_back(degrees, (int32_t)((int64_t)S * q / nth),
                              (int32_t)((int64_t)S * (q + 1) / nth));
        for (std::thread &t : pool) t.join();
    }
    std::vector<int32_t> order((size_t)S);
    for (int32_t j = 0; j < S; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return deg[a] != deg[b] ? deg[a] > deg[b] : a < b;
    });
    std::vector<int32_t> colour((size_t)S, -1), used;
    int32_t k = 0;
    for (int32_t j : order) {
        for_conflicts(j, [&](int32_t x) {
            if (colour[x] >= 0) used[colour[x]] = j;
        });
        int32_t c = 0;
        while (c < k && used[c] == j) ++c;
        if (c == k) {
            used.push_back(-1);
            ++k;
        }
        colour[j] = c;
    }
    f->k = k;
    f->colour = colour;
    f->class_ptr.assign((size_t)k + 1, 0);
    for (int32_t j = 0; j < S; ++j) f->class_ptr[(size_t)colour[j] + 1]++;
    for (int32_t c = 0; c < k; ++c) f->class_ptr[(size_t)c + 1] += f->class_ptr[c];
    f->class_elems.assign((size_t)S, 0);
    std::vector<int32_t> fill(f->class_ptr.begin(), f->class_ptr.end() - 1);
    for (int32_t j = 0; j < S; ++j) f->class_elems[(size_t)fill[colour[j]]++] = j;
    f->coloured = true;
    if (n_colours) *n_colours = k;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_colour_get(const gom_fos *f, int32_t *colour_of_set, int32_t *class_ptr,
                              int32_t *class_elems) {
    if (!f) return fail(GOM_E_ARG, "gom_colour_get: null fos");
    if (!f->coloured) return fail(GOM_E_STATE, "gom_colour_get: FOS not coloured");
    if (colour_of_set) std::copy(f->colour.begin(), f->colour.end(), colour_of_set);
    if (class_ptr) std::copy(f->class_ptr.begin(), f->class_ptr.end(), class_ptr);
    if (class_elems) std::copy(f->class_elems.begin(), f->class_elems.end(), class_elems);
    return GOM_OK;
}

// ------------------------------------------------------------------------------------------
// State
// ------------------------------------------------------------------------------------------
static int check_state_args(const mc_graph *g, const gom_fos *f, int32_t pop) {
    if (!g || !f) return fail(GOM_E_ARG, "null graph or fos");
    if (f->n_vars != g->n) return fail(GOM_E_ARG, "FOS built for another graph");
    if (!f->coloured) return fail(GOM_E_STATE, "FOS not coloured (call gom_colour first)");
    if (pop < 2 || pop > GOM_MAX_POP)
        return fail(GOM_E_RANGE, "population %d outside [2, %d]", pop, GOM_MAX_POP);
    return GOM_OK;
}

extern "C" int gom_state_bytes(const mc_graph *g, const gom_fos *f, int32_t pop, size_t *bytes) {
    GUARD_BEGIN
    int rc = check_state_args(g, f, pop);
    if (rc) return rc;
    if (!bytes) return fail(GOM_E_ARG, "gom_state_bytes: null output");
    if (g->n >= kMaxVertexSmall)
        return fail(GOM_E_RANGE, "gom_state_bytes: at most %d vertices", kMaxVertexSmall - 1);
    Records R;
    rc = build_records(*g, *f, f->max_set == 1, R);
    if (rc) return rc;
    const CoopSets CS = coop_sets(*f, f->max_set == 1);
    const int64_t sw_words = swar_eligible(*g, *f) ? (int64_t)kSwRows * swar_stride(f->n_sets) : 0;
    *bytes = make_layout(g->n, g->m, f->n_sets, f->k, pop, (int64_t)R.words.size(),
                         (int64_t)CS.pos.size(), sw_words, (int64_t)CS.smap.size()).total;
    return GOM_OK;
    GUARD_END
}

static std::vector<int32_t> class_order(const gom_state *s, int32_t gen) {
    std::vector<int32_t> perm((size_t)s->k);
    for (int32_t c = 0; c < s->k; ++c) perm[c] = c;
    if (s->order == GOM_ORDER_RANDOM)
        for (int32_t t = s->k - 1; t >= 1; --t) {
            const U32x4 r = philox(s->seed, (uint32_t)gen, kOrderStream, (uint32_t)t, 0u);
            const int32_t x = (int32_t)(((uint64_t)r.x * (uint64_t)(t + 1)) >> 32);
            std::swap(perm[t], perm[x]);
        }
    return perm;
}

// Sampled kernel timing: every `timing`-th sweep launch gets a pair of events that the launch
// records with its own dispatch.
static int timing_events(gom_state *s, KernelEvents *ev) {
    *ev = KernelEvents{};
    if (!s->timing) return GOM_OK;
    if (s->sweep_launches++ % s->timing != 0) return GOM_OK;
    if (s->tev_used + 2 > s->tev.size()) {
        if (s->tev.size() < (size_t)(1 << 15)) {
            const size_t grow = s->tev.size() ? s->tev.size() : 256;
            for (size_t q = 0; q < grow; ++q) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                s->tev.push_back(e);
            }
        } else {
            // Pool full: fold the recorded pairs into the running total and reuse them.
            for (size_t q = 0; q + 1 < s->tev_used; q += 2) {
                float ms = 0.f;
                HIP_TRY(hipEventSynchronize(s->tev[q + 1]));
                HIP_TRY(hipEventElapsedTime(&ms, s->tev[q], s->tev[q + 1]));
                s->t_ms += ms;
                s->t_launches++;
            }
            s->tev_used = 0;
        }
    }
    ev->start = s->tev[s->tev_used++];
    ev->stop = s->tev[s->tev_used++];
    return GOM_OK;
}

// Enqueue generation `gen` (Algorithm 3): every colour class in the generation's order, then
// the epilogue.  Kernels skip their work when the elitist has already reached `target`.
// Device address of the state's forced-improvement records (DevState::fi_at).
static uint32_t *fi_at_ptr(const gom_state *s) {
    return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(s->d_st) +
                                        offsetof(DevState, fi_at));
}

static ResidentCtx resident_ctx(const gom_state *s, int64_t target) {
    ResidentCtx r{};
    r.P = s->d_P;
    r.rows = s->d_rows;
    r.stripes = s->d_stripes;
    r.st = s->d_st;
    r.roff = s->d_roff;
    r.recs = s->d_recs;
    r.class_rec = s->d_crec;
    r.class_ptr = s->d_cptr;
    r.seed = s->seed;
    r.target = target;
    r.n = s->n;
    r.N = s->N;
    r.k = s->k;
    r.always = s->rule == GOM_NEUTRAL_ALWAYS;
    r.row_words = (s->n + 63) / 64;
    r.fi = s->fi ? 1 : 0;
    r.E = s->d_E;
    r.fi_at = fi_at_ptr(s);
    return r;
}

static EpilogueArgs epilogue_args(const gom_state *s, int64_t target, bool rows) {
    EpilogueArgs e{};
    e.P = s->d_P;
    e.O = s->d_O;
    e.rows = rows ? s->d_rows : nullptr;
    e.E = s->d_E;
    e.fit = s->d_fit;
    e.st = s->d_st;
    e.stripes = s->d_stripes;
    e.target = target;
    e.n = s->n;
    e.N = s->N;
    e.mode = kEpiGeneration;
    e.row_words = (s->n + 63) / 64;
    e.fi = s->fi ? 1 : 0;
    return e;
}

static int enqueue_epilogue(gom_state *s, int64_t target, hipStream_t st, bool rows) {
    HIP_TRY(launch_epilogue(epilogue_args(s, target, rows), st));
    return GOM_OK;
}

// Class sweeps for order positions [t0, t1) of generation `gen` under the per-class schedules
// (bit-sliced when chosen, else class launch).
// Class c has no set for the block-cooperative or split sweeps.
static bool nl_coop_free(const gom_state *s, int32_t c) {
    return s->coop_ptr[2 * (size_t)c + 2] == s->coop_ptr[2 * (size_t)c] && !s->split[(size_t)c];
}

// Classes the general bit-sliced sweep takes (general FOS, population <= 64): sets of at most
// kGsMaxMembers members, per-set sums of |w| within kGsMaxWeightSum, |w| within
// kGsMaxWeightBits bits, no set left to a block-cooperative sweep, at least gs_min_sets sets.
// Records the largest |w|'s bit count per class (0: not taken); true when some class is taken.
static bool gs_select(gom_state *s) {
    s->gs_wbits.assign((size_t)s->k, 0);
    if (s->univariate || s->N > 64) return false;
    bool any = false;
    for (int32_t c = 0; c < s->k; ++c) {
        int bits = 1;
        while (bits < 62 && (s->class_wmax[c] >> bits) != 0) ++bits;
        const bool ok = s->class_members[c] <= kGsMaxMembers &&
                        s->class_wsum[c] <= kGsMaxWeightSum && bits <= kGsMaxWeightBits &&
                        nl_coop_free(s, c) &&
                        s->class_ptr[(size_t)c + 1] - s->class_ptr[c] >= s->gs_min_sets;
        s->gs_wbits[c] = ok ? (int8_t)bits : 0;
        any |= ok;
    }
    return any;
}

// The generation-wide fields of a class sweep's arguments.
static SweepArgs sweep_args(const gom_state *s, int32_t gen, int64_t target, bool forced) {
    SweepArgs a{};
    a.mode = forced ? kSweepFi : (s->fi ? kSweepGomTrack : kSweepGom);
    a.E = s->d_E;
    a.P = s->d_P;
    a.O = s->d_O;
    a.stripes = s->d_stripes;
    a.st = s->d_st;
    a.roff = s->d_roff;
    a.recs = s->d_recs;
    a.sw = s->d_sw;
    a.sw_stride = s->sw_stride;
    a.fi_at = fi_at_ptr(s);
    a.seed = s->seed;
    a.target = target;
    a.N = s->N;
    a.gen = gen;
    a.always = s->rule == GOM_NEUTRAL_ALWAYS;
    return a;
}

// Every class of a whole generation in one cooperative launch of the fused bit-sliced sweep.
static int enqueue_fused_generation(gom_state *s, const std::vector<int32_t> &perm, int32_t gen,
                                    int64_t target, hipStream_t st) {
    FusedArgs f{};
    f.a = sweep_args(s, gen, target, false);
    f.dep = s->d_fdep;
    f.flags = s->d_fflags;
    f.epoch = ++s->fused_epoch;
    if (f.epoch == 0) {
        // after 2^32 launches the stamps wrap: start the flags again from zero
        HIP_TRY(hipMemsetAsync(s->d_fflags, 0, sizeof(uint32_t) * (size_t)s->k * s->fused_grid,
                               st));
        f.epoch = s->fused_epoch = 1;
    }
    f.k = s->k;
    f.grid = s->fused_grid;
    for (int32_t t = 0; t < s->k; ++t) {
        const int32_t c = perm[(size_t)t];
        f.order[t] = c;
        f.cbase[c] = s->class_ptr[c];
        f.csize[c] = s->class_ptr[(size_t)c + 1] - s->class_ptr[c];
        f.clen[c] = s->fused_clen[(size_t)c];
    }
    KernelEvents ev;
    int rc = timing_events(s, &ev);
    if (rc) return rc;
    if (ev.start) HIP_TRY(hipEventRecord(ev.start, st));
    HIP_TRY(launch_uni_swar_fused(f, s->partition, s->fused_narrow, st));
    if (ev.stop) HIP_TRY(hipEventRecord(ev.stop, st));
    return GOM_OK;
}

static int enqueue_class_range(gom_state *s, const std::vector<int32_t> &perm, int32_t gen,
                               int32_t t0, int32_t t1, int64_t target, hipStream_t st,
                               bool forced = false) {
    SweepArgs a = sweep_args(s, gen, target, forced);
    for (int32_t t = t0; t < t1; ++t) {
        const int32_t c = perm[t];
        a.cls = c;
        a.fi_pos = t;
        a.cbase = s->class_ptr[c];
        a.rbase = s->class_rec[c].x;
        a.rstride = s->class_rec[c].y;
        a.csize = s->class_ptr[(size_t)c + 1] - s->class_ptr[c];
        KernelEvents ev;
        int rc = forced ? GOM_OK : timing_events(s, &ev);
        if (rc) return rc;
        const int32_t nl = s->coop_ptr[2 * (size_t)c + 2] - s->coop_ptr[2 * (size_t)c];
        a.coop = nl > 0 ? 1 : 0;
        // small general sets swept with every solution of a wave (64 lanes) take the staged
        // evaluation: the set's record and words in two rounds of loads
        const bool staged = s->staged_use && !forced && !s->univariate && s->N > 32 &&
                            s->class_members[c] <= kBclMaxMembers &&
                            s->class_entries[c] <= kBclMaxEntries && nl_coop_free(s, c);
        if (s->sched == GOM_SCHED_BITSLICED && !forced && s->univariate)
            HIP_TRY(launch_uni_swar_sweep(a, s->partition, s->swar_narrow, s->max_grid, st, ev));
        else if (s->sched == GOM_SCHED_BITSLICED && !forced && s->gs_wbits[c])
            HIP_TRY(launch_gen_swar_sweep(a, s->class_members[c], s->gs_wbits[c], s->max_grid,
                                          st, ev));
        else if (staged)
            HIP_TRY(launch_class_sweep_staged(a, s->max_grid, s->sweep_threads, st, ev));
        else
            HIP_TRY(launch_class_sweep(a, s->univariate ? 0 : 1,
                                       s->class_entries[c] <= kShortRecordEntries, s->max_grid,
                                       s->sweep_threads, st, ev));
        if (s->split[c]) {  // every large set of the class in one split sweep
            SweepArgs b = a;
            b.smap = s->d_smap + s->smap_ptr[c];
            b.n_smap = s->smap_ptr[(size_t)c + 1] - s->smap_ptr[c];
            b.split_D = s->d_split_D;
            b.split_delta = s->d_split_delta;
            b.split_sel = s->d_split_sel;
            HIP_TRY(launch_split_sweep(b, st));
            continue;
        }
        for (int grp = 0; grp < 2; ++grp) {
            const size_t q = 2 * (size_t)c + grp;
            SweepArgs b = a;
            b.n_large = s->coop_ptr[q + 1] - s->coop_ptr[q];
            if (b.n_large == 0) continue;
            b.large_pos = s->d_coop + s->coop_ptr[q];
            b.coop_cap = s->coop_max[q];
            HIP_TRY(launch_large_set_sweep(b, s->coop_max[q], grp ? 1024 : kCoopSmallBlock, st));
        }
    }
    return GOM_OK;
}

static int enqueue_generation(gom_state *s, int32_t gen, int64_t target, hipStream_t st) {
    const std::vector<int32_t> perm = class_order(s, gen);
    if (s->open_next >= 0) {
        // finish a generation left open by gom_debug_stop_after_class; its offspring are in
        // the O planes, so the rest runs class by class
        int rc = enqueue_class_range(s, perm, gen, s->open_next, s->k, target, st);
        if (rc == GOM_OK && s->fi) rc = enqueue_class_range(s, perm, gen, 0, s->k, target, st, true);
        if (rc) return rc;
        s->open_next = -1;
        return enqueue_epilogue(s, target, st, false);
    }
    if (s->sched == GOM_SCHED_RESIDENT) {
        ResidentArgs r{};
        r.c = resident_ctx(s, target);
        r.c.gen = gen;
        for (int32_t t = 0; t < s->k; ++t) r.order[t] = (uint16_t)perm[t];
        KernelEvents ev;
        int rc = timing_events(s, &ev);
        if (rc) return rc;
        HIP_TRY(launch_resident_sweep(r, s->univariate ? 0 : 1, s->resident_plds, st, ev));
        return enqueue_epilogue(s, target, st, true);
    }
    if (s->sched == GOM_SCHED_BITSLICED && s->fused_ok && s->fused_use && !s->fi) {
        const int rc = enqueue_fused_generation(s, perm, gen, target, st);
        if (rc) return rc;
        return enqueue_epilogue(s, target, st, false);
    }
    int rc = enqueue_class_range(s, perm, gen, 0, s->k, target, st);
    // forced improvement: the classes again, with the elitist as donor
    if (rc == GOM_OK && s->fi) rc = enqueue_class_range(s, perm, gen, 0, s->k, target, st, true);
    if (rc) return rc;
    return enqueue_epilogue(s, target, st, false);
}

// InitializePopulation (Algorithm 3), full fitness of every solution, initial elitist.
static hipError_t enqueue_initial_population(gom_state *s, hipStream_t st) {
    hipError_t e = launch_init_population(s->d_P, s->d_O, s->d_fit, s->d_st, s->d_stripes, s->n,
                                          s->N, s->seed, st);
    if (e == hipSuccess)
        e = launch_full_fitness(s->d_P, s->d_eu, s->d_ev, s->d_ew, s->m, s->N, s->d_stripes, st);
    if (e != hipSuccess) return e;
    EpilogueArgs ea{};
    ea.P = s->d_P;
    ea.O = s->d_O;
    ea.E = s->d_E;
    ea.fit = s->d_fit;
    ea.st = s->d_st;
    ea.stripes = s->d_stripes;
    ea.target = INT64_MAX;
    ea.n = s->n;
    ea.N = s->N;
    ea.mode = kEpiInit;
    e = launch_epilogue(ea, st);
    if (e == hipSuccess) {
        s->g_host = 0;
        s->g_base = 0;
        s->attempted_base = 0;
        s->open_next = -1;
    }
    return e;
}

static int auto_schedule(const gom_state *s) {
    if (s->resident_ok && s->n <= kResidentAutoMaxVertices) return GOM_SCHED_RESIDENT;
    // (general FOS: only classes of at least gs_min_sets sets take the bit-sliced sweep, the
    // others the class sweep, so an instance with such a class gains and none loses)
    if (s->bitsliced_ok && !s->fi) return GOM_SCHED_BITSLICED;
    return GOM_SCHED_CLASS_LAUNCH;
}

// The bit-sliced sweep's 32-bit block counters suffice: a block sums the changes of at most
// 256 threads x (sets per thread) flips per solution, each at most the largest per-vertex
// |weight| sum.
static bool swar_narrow_ok(const gom_state *s) {
    const int64_t per_thread =
        ((int64_t)s->max_class + (int64_t)s->max_grid * kSwarThreads - 1) /
        ((int64_t)s->max_grid * kSwarThreads);
    return s->swar_abs * kSwarThreads * per_thread < ((int64_t)1 << 31);
}

// pinned_host: the run-scalar read-back buffer is pinned host memory (hipHostMalloc); else
// ordinary host memory, so that the state's creation allocates nothing through HIP.
static int state_init(const mc_graph *g, const gom_fos *f, int32_t pop, uint64_t seed,
                      int neutral_rule, int class_order_kind, void *dev_arena, size_t arena_bytes,
                      void *stream, bool pinned_host, gom_state **out) {
    int rc = check_state_args(g, f, pop);
    if (rc) return rc;
    if (!dev_arena || !out) return fail(GOM_E_ARG, "gom_state_init: null arena or output");
    if (neutral_rule != GOM_NEUTRAL_PAPER && neutral_rule != GOM_NEUTRAL_ALWAYS)
        return fail(GOM_E_ARG, "gom_state_init: unknown neutral rule %d", neutral_rule);
    if (class_order_kind != GOM_ORDER_RANDOM && class_order_kind != GOM_ORDER_FIXED)
        return fail(GOM_E_ARG, "gom_state_init: unknown class order %d", class_order_kind);
    if ((reinterpret_cast<uintptr_t>(dev_arena) & 255) != 0)
        return fail(GOM_E_NOMEM, "gom_state_init: arena must be 256-byte aligned");
    if (g->n >= kMaxVertexSmall)
        return fail(GOM_E_RANGE, "gom_state_init: at most %d vertices", kMaxVertexSmall - 1);
    Records R;
    rc = build_records(*g, *f, f->max_set == 1, R);
    if (rc) return rc;
    const CoopSets CS = coop_sets(*f, f->max_set == 1);
    int64_t swar_abs = 0;
    const bool swar = swar_eligible(*g, *f, &swar_abs);
    const std::vector<int32_t> SW = swar ? build_swar(*g, *f) : std::vector<int32_t>();
    const Layout L = make_layout(g->n, g->m, f->n_sets, f->k, pop, (int64_t)R.words.size(),
                                 (int64_t)CS.pos.size(), (int64_t)SW.size(),
                                 (int64_t)CS.smap.size());
    if (arena_bytes < L.total)
        return fail(GOM_E_NOMEM, "gom_state_init: arena has %zu bytes, needs %zu", arena_bytes,
                    L.total);
    hipStream_t st = (hipStream_t)stream;
    auto *s = new gom_state;
    s->n = g->n;
    s->m = g->m;
    s->N = pop;
    s->n_sets = f->n_sets;
    s->k = f->k;
    s->seed = seed;
    s->rule = neutral_rule;
    s->order = class_order_kind;
    s->univariate = f->max_set == 1;
    s->max_set = f->max_set;
    s->class_ptr = f->class_ptr;
    for (int32_t c = 0; c < f->k; ++c)
        s->max_class = std::max(s->max_class, f->class_ptr[(size_t)c + 1] - f->class_ptr[c]);
    s->arena = (char *)dev_arena;
    s->L = L;
    s->d_st = (DevState *)(s->arena + L.st);
    s->d_fit = (int64_t *)(s->arena + L.fit);
    s->d_stripes = (Stripe *)(s->arena + L.stripes);
    s->d_E = (uint64_t *)(s->arena + L.E);
    s->d_P = (uint64_t *)(s->arena + L.P);
    s->d_O = (uint64_t *)(s->arena + L.O);
    s->d_rows = (uint64_t *)(s->arena + L.rows);
    s->d_cptr = (int32_t *)(s->arena + L.cptr);
    s->d_eu = (int32_t *)(s->arena + L.eu);
    s->d_ev = (int32_t *)(s->arena + L.ev);
    s->d_ew = (int32_t *)(s->arena + L.ew);
    s->d_roff = (int32_t *)(s->arena + L.roff);
    s->d_recs = (int32_t *)(s->arena + L.recs);
    s->d_crec = (int2 *)(s->arena + L.crec);
    s->class_rec = R.class_rec;
    s->class_entries = R.class_entries;
    s->class_members = R.class_members;
    s->class_wsum = R.class_wsum;
    s->class_wmax = R.class_wmax;
    s->coop_ptr = CS.ptr;
    s->coop_max = CS.max_members;
    s->d_coop = (int32_t *)(s->arena + L.coop);
    s->d_sw = (int32_t *)(s->arena + L.sw);
    s->split = CS.split;
    s->smap_ptr = CS.smap_ptr;
    s->d_smap = (int4 *)(s->arena + L.smap);
    s->d_split_D = (uint64_t *)(s->arena + L.split);
    s->d_split_delta = (int64_t *)(s->arena + L.split + (size_t)kSplitBelow * 64 * 8);
    s->d_split_sel = (int32_t *)(s->arena + L.split + (size_t)kSplitBelow * 64 * 16);
    s->sw_stride = swar_stride(f->n_sets);
    s->d_fdep = (int4 *)(s->arena + L.fdep);
    s->d_fflags = (uint32_t *)(s->arena + L.fflags);
    auto cleanup = [&](int code) {
        gom_state_free(s);
        return code;
    };
    auto h2d = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    if (pinned_host) {
        e = hipHostMalloc((void **)&s->h_st, 2 * sizeof(DevState), hipHostMallocDefault);
    } else {
        s->h_st = new DevState[2];
        s->h_st_pinned = false;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->chunk_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->chunk_ev[1], hipEventDisableTiming);
    if (e == hipSuccess) e = h2d(s->d_eu, g->eu.data(), sizeof(int32_t) * (size_t)g->m);
    if (e == hipSuccess) e = h2d(s->d_ev, g->ev.data(), sizeof(int32_t) * (size_t)g->m);
    if (e == hipSuccess) e = h2d(s->d_ew, g->ew.data(), sizeof(int32_t) * (size_t)g->m);
    if (e == hipSuccess)
        e = h2d(s->d_cptr, f->class_ptr.data(), sizeof(int32_t) * f->class_ptr.size());
    if (e == hipSuccess) {
        int dev = 0, lds_max = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        s->lds_max = (size_t)lds_max;
        s->resident_ok = e == hipSuccess && s->k <= kResidentMaxClasses &&
                         resident_lds_bytes(s->n, false) <= s->lds_max;
        s->resident_plds = s->resident_ok && resident_lds_bytes(s->n, true) <= s->lds_max;
        s->swar_uni = swar;
        s->bitsliced_ok = swar || gs_select(s);
        s->swar_abs = swar_abs;
        s->swar_narrow = swar && swar_narrow_ok(s);
        s->partition = s->univariate && f->n_sets == g->n;
        s->sched = auto_schedule(s);
    }
    if (e == hipSuccess) e = h2d(s->d_roff, R.roff.data(), sizeof(int32_t) * R.roff.size());
    if (e == hipSuccess) e = h2d(s->d_recs, R.words.data(), sizeof(int32_t) * R.words.size());
    if (e == hipSuccess)
        e = h2d(s->d_crec, R.class_rec.data(), sizeof(int2) * R.class_rec.size());
    if (e == hipSuccess) e = h2d(s->d_coop, CS.pos.data(), sizeof(int32_t) * CS.pos.size());
    if (e == hipSuccess) e = h2d(s->d_sw, SW.data(), sizeof(int32_t) * SW.size());
    if (e == hipSuccess) e = h2d(s->d_smap, CS.smap.data(), sizeof(int4) * CS.smap.size());
    std::vector<int4> fdep;
    if (e == hipSuccess && swar && f->k <= kFusedMaxClasses) {
        // the fused form of the bit-sliced sweep: one cooperative launch per generation
        int grid = 0;
        e = fused_swar_grid(&grid);
        // no more blocks than a thread per set of the largest class needs: chunks of at least
        // a block's width keep the dependency ranges short
        grid = std::min<int64_t>(grid, ((int64_t)s->max_class + kSwarThreads - 1) / kSwarThreads);
        if (e == hipSuccess && grid >= 1 && fused_deps(*g, *f, grid, s->fused_clen, fdep)) {
            int64_t per_thread = 0;  // sets a thread sweeps per generation
            for (int32_t c = 0; c < f->k; ++c)
                per_thread += (s->fused_clen[(size_t)c] + kSwarThreads - 1) / kSwarThreads;
            s->fused_narrow = swar_abs * kSwarThreads * per_thread < ((int64_t)1 << 31);
            s->fused_grid = grid;
            s->fused_ok = true;
            e = h2d(s->d_fdep, fdep.data(), sizeof(int4) * fdep.size());
            if (e == hipSuccess)
                e = hipMemsetAsync(s->d_fflags, 0, sizeof(uint32_t) * (size_t)f->k * grid, st);
        }
    }
    if (e == hipSuccess && !CS.smap.empty())  // the split sweep's scratch starts cleared
        e = hipMemsetAsync(s->arena + L.split, 0, kSplitScratchBytes, st);
    if (e == hipSuccess) e = enqueue_initial_population(s, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host staging buffers die below
    if (e != hipSuccess)
        return cleanup(fail(GOM_E_DEVICE, "gom_state_init: %s", hipGetErrorString(e)));
    *out = s;
    return GOM_OK;
}

extern "C" int gom_state_init(const mc_graph *g, const gom_fos *f, int32_t pop, uint64_t seed,
                              int neutral_rule, int class_order_kind, void *dev_arena,
                              size_t arena_bytes, void *stream, gom_state **out) {
    GUARD_BEGIN
    return state_init(g, f, pop, seed, neutral_rule, class_order_kind, dev_arena, arena_bytes,
                      stream, true, out);
    GUARD_END
}

// Devices whose static arena holds a live state (one at a time per device).
static std::mutex g_static_mu;
static std::vector<bool> g_static_busy;

extern "C" int gom_state_init_static(const mc_graph *g, const gom_fos *f, int32_t pop,
                                     uint64_t seed, int neutral_rule, int class_order_kind,
                                     void *stream, gom_state **out) {
    GUARD_BEGIN
    if (!out) return fail(GOM_E_ARG, "gom_state_init_static: null output");
    size_t need = 0;
    int rc = gom_state_bytes(g, f, pop, &need);
    if (rc) return rc;
    if (need > kStaticArenaBytes)
        return fail(GOM_E_RANGE, "gom_state_init_static: the state needs %zu bytes, the static "
                    "arena holds %zu", need, (size_t)kStaticArenaBytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    void *arena = nullptr;
    HIP_TRY(static_arena_address(&arena));
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_busy.size() <= (size_t)dev) g_static_busy.resize((size_t)dev + 1, false);
        if (g_static_busy[(size_t)dev])
            return fail(GOM_E_STATE, "gom_state_init_static: device %d's static arena holds a "
                        "live state (free it first)", dev);
        g_static_busy[(size_t)dev] = true;
    }
    gom_state *s = nullptr;
    rc = state_init(g, f, pop, seed, neutral_rule, class_order_kind, arena, kStaticArenaBytes,
                    stream, false, &s);
    if (rc) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[(size_t)dev] = false;
        return rc;
    }
    s->static_dev = dev;
    *out = s;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_state_reseed(gom_state *s, uint64_t seed, void *stream) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_state_reseed: null state");
    s->seed = seed;
    HIP_TRY(enqueue_initial_population(s, (hipStream_t)stream));
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_generation(gom_state *s, void *stream) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_generation: null state");
    int rc = enqueue_generation(s, s->g_host, INT64_MAX, (hipStream_t)stream);
    if (rc) return rc;
    s->g_host++;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_debug_stop_after_class(gom_state *s, int32_t class_position, void *stream) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_debug_stop_after_class: null state");
    if (class_position < 0 || class_position >= s->k)
        return fail(GOM_E_RANGE, "gom_debug_stop_after_class: position %d outside [0, %d)",
                    class_position, s->k);
    const int32_t from = s->open_next >= 0 ? s->open_next : 0;
    if (class_position < from)
        return fail(GOM_E_STATE,
                    "gom_debug_stop_after_class: the open generation is already past position %d",
                    class_position);
    const std::vector<int32_t> perm = class_order(s, s->g_host);
    int rc = enqueue_class_range(s, perm, s->g_host, from, class_position + 1, INT64_MAX,
                                 (hipStream_t)stream);
    if (rc) return rc;
    s->open_next = class_position + 1;
    return GOM_OK;
    GUARD_END
}

static int read_scalars(gom_state *s, hipStream_t st, DevState *h);

// Passes of the colouring-parallel local search over the O planes: one k_ls_sweep launch per
// colour class in ascending class index, then a read-back of the flip flag; the passes stop
// after one that flipped nothing, or at max_passes.
static int ls_pass_loop(gom_state *s, int32_t max_passes, hipStream_t st, int32_t *passes_out) {
    uint32_t *d_any = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(s->d_st) +
                                                   offsetof(DevState, ls_any));
    SweepArgs a{};
    a.O = s->d_O;
    a.stripes = s->d_stripes;
    a.st = s->d_st;
    a.roff = s->d_roff;
    a.recs = s->d_recs;
    a.N = s->N;
    a.ls_any = d_any;
    int32_t passes = 0;
    while (passes < max_passes) {
        HIP_TRY(hipMemsetAsync(d_any, 0, sizeof(uint32_t), st));
        for (int32_t c = 0; c < s->k; ++c) {
            a.cls = c;
            a.cbase = s->class_ptr[c];
            a.rbase = s->class_rec[c].x;
            a.rstride = s->class_rec[c].y;
            a.csize = s->class_ptr[(size_t)c + 1] - s->class_ptr[c];
            HIP_TRY(launch_ls_sweep(a, s->max_grid, st));
        }
        HIP_TRY(hipMemcpyAsync(&s->h_st[0].ls_any, d_any, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ++passes;
        if (!s->h_st[0].ls_any) break;
    }
    *passes_out = passes;
    return GOM_OK;
}

// Colouring-parallel local search (declared in gom.h): the pass loop above, then the
// generation-end epilogue without a generation count.
extern "C" int gom_local_search(gom_state *s, int32_t max_passes, void *stream,
                                int32_t *passes_out) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_local_search: null state");
    if (max_passes < 0) return fail(GOM_E_ARG, "gom_local_search: max_passes %d < 0", max_passes);
    if (!s->univariate)
        return fail(GOM_E_STATE, "gom_local_search: the state's FOS is not univariate");
    if (s->open_next >= 0)
        return fail(GOM_E_STATE, "gom_local_search: a generation is open");
    hipStream_t st = (hipStream_t)stream;
    int32_t passes = 0;
    int rc = ls_pass_loop(s, max_passes, st, &passes);
    if (rc) return rc;
    EpilogueArgs e = epilogue_args(s, INT64_MAX, false);
    e.mode = kEpiLocalSearch;
    HIP_TRY(launch_epilogue(e, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (passes_out) *passes_out = passes;
    return GOM_OK;
    GUARD_END
}

// Iterated local search (declared in gom.h): per round one k_perturb launch (the flips go
// into O, their gains into a stripe), the pass loop, and the epilogue in its iterated mode
// (each solution keeps the round's result unless its fitness fell, then P <- O).
extern "C" int gom_iterated_local_search(gom_state *s, int32_t round0, int32_t rounds,
                                         int32_t flips, int32_t max_passes, void *stream,
                                         int32_t *passes_out) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_iterated_local_search: null state");
    if (round0 < 0 || rounds < 0 || (int64_t)round0 + rounds > kMaxPerturbRounds)
        return fail(GOM_E_ARG, "gom_iterated_local_search: rounds [%d, %d + %d) outside "
                    "[0, 2^27)", round0, round0, rounds);
    if (flips < 0 || flips > 64)
        return fail(GOM_E_ARG, "gom_iterated_local_search: flips %d outside 0..64", flips);
    if (max_passes < 0)
        return fail(GOM_E_ARG, "gom_iterated_local_search: max_passes %d < 0", max_passes);
    if (!s->univariate)
        return fail(GOM_E_STATE, "gom_iterated_local_search: the state's FOS is not univariate");
    if (s->open_next >= 0)
        return fail(GOM_E_STATE, "gom_iterated_local_search: a generation is open");
    hipStream_t st = (hipStream_t)stream;
    int rc = read_scalars(s, st, &s->h_st[0]);
    if (rc) return rc;
    PerturbArgs pa{};
    pa.P = s->d_P;
    pa.O = s->d_O;
    pa.recs = s->d_recs;
    pa.roff = s->d_roff;
    pa.stripes = s->d_stripes;
    pa.seed = s->seed;
    pa.gen = s->h_st[0].generation;
    pa.flips = flips;
    pa.n_sets = s->n_sets;
    pa.N = s->N;
    EpilogueArgs e = epilogue_args(s, INT64_MAX, false);
    e.mode = kEpiIterated;
    int32_t total = 0;
    for (int32_t r = round0; r < round0 + rounds; ++r) {
        pa.round = r;
        HIP_TRY(launch_perturb(pa, st));
        int32_t passes = 0;
        rc = ls_pass_loop(s, max_passes, st, &passes);
        if (rc) return rc;
        total += passes;
        HIP_TRY(launch_epilogue(e, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (passes_out) *passes_out = total;
    return GOM_OK;
    GUARD_END
}

static int check_stall(const DevState &h) {
    if (h.stall)
        return fail(GOM_E_DEVICE, "a dependency wait of the fused bit-sliced sweep gave up; the "
                    "state is not valid");
    return GOM_OK;
}

static int read_scalars(gom_state *s, hipStream_t st, DevState *h) {
    HIP_TRY(hipMemcpyAsync(h, s->d_st, sizeof(DevState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return check_stall(*h);
}

// Fitness and counters of the state.  While a generation is open the running values are the
// stored ones plus what the class sweeps have added to the stripes so far.
static int read_fitness_counters(gom_state *s, hipStream_t st, int64_t *fit, DevState *h,
                                 int64_t counters[3]) {
    HIP_TRY(hipMemcpyAsync(fit, s->d_fit, sizeof(int64_t) * (size_t)s->N, hipMemcpyDeviceToHost,
                           st));
    std::vector<Stripe> stripes;
    if (s->open_next >= 0) {
        stripes.resize(kStripes);
        HIP_TRY(hipMemcpyAsync(stripes.data(), s->d_stripes, sizeof(Stripe) * kStripes,
                               hipMemcpyDeviceToHost, st));
    }
    int rc = read_scalars(s, st, h);
    if (rc) return rc;
    counters[0] =
        s->attempted_base + (int64_t)s->N * s->n_sets * (int64_t)(h->generation - s->g_base);
    counters[1] = h->evaluated;
    counters[2] = h->accepted;
    if (s->open_next >= 0) {
        for (const Stripe &sp : stripes) {
            for (int32_t i = 0; i < s->N; ++i) fit[i] += sp.fit[i];
            counters[1] += (int64_t)sp.evaluated;
            counters[2] += (int64_t)sp.accepted;
        }
        const std::vector<int32_t> perm = class_order(s, s->g_host);
        for (int32_t t = 0; t < s->open_next; ++t)
            counters[0] += (int64_t)s->N *
                           (s->class_ptr[(size_t)perm[t] + 1] - s->class_ptr[perm[t]]);
    }
    return GOM_OK;
}

extern "C" int gom_run_to_target(gom_state *s, int64_t target, int32_t max_generations,
                                 void *stream, gom_result *out) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_run_to_target: null state");
    if (s->open_next >= 0)
        return fail(GOM_E_STATE, "gom_run_to_target: a generation is open (finish it with "
                                 "gom_generation)");
    hipStream_t st = (hipStream_t)stream;
    int rc = read_scalars(s, st, &s->h_st[0]);
    if (rc) return rc;
    s->g_host = s->h_st[0].generation;
    const int32_t g0 = s->g_host;
    constexpr int32_t kChunk = 4;
    if (s->h_st[0].elite_fitness < target && s->g_host < max_generations) {
        int32_t issued = s->g_host;
        int slot = 0, prev = -1;
        for (;;) {
            const int32_t n = std::min(kChunk, max_generations - issued);
            int cur = -1;
            if (n > 0) {
                for (int32_t t = 0; t < n; ++t) {
                    rc = enqueue_generation(s, issued + t, target, st);
                    if (rc) return rc;
                }
                issued += n;
                cur = slot;
                HIP_TRY(hipMemcpyAsync(&s->h_st[cur], s->d_st, sizeof(DevState),
                                       hipMemcpyDeviceToHost, st));
                HIP_TRY(hipEventRecord(s->chunk_ev[cur], st));
                slot ^= 1;
            }
            if (prev >= 0) {
                HIP_TRY(hipEventSynchronize(s->chunk_ev[prev]));
                rc = check_stall(s->h_st[prev]);
                if (rc) return rc;
                if (s->h_st[prev].elite_fitness >= target) break;
            }
            if (cur < 0) break;
            prev = cur;
        }
    }
    DevState fin;
    rc = read_scalars(s, st, &fin);
    if (rc) return rc;
    s->g_host = fin.generation;
    if (out) {
        out->generations = fin.generation - g0;
        out->reached = fin.elite_fitness >= target;
        out->best = fin.elite_fitness;
        out->attempted =
            s->attempted_base + (int64_t)s->N * s->n_sets * (int64_t)(fin.generation - s->g_base);
        out->evaluated = fin.evaluated;
        out->accepted = fin.accepted;
    }
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_state_read(gom_state *s, void *stream, uint8_t *genes, int64_t *fitness,
                              uint8_t *elite, int64_t *elite_fitness, int32_t *generation,
                              int64_t *counters) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_state_read: null state");
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint64_t> P, E;
    int64_t fit[GOM_MAX_POP];
    if (genes) {
        // the offspring planes while a generation is open (equal to P otherwise)
        P.resize((size_t)s->n);
        HIP_TRY(hipMemcpyAsync(P.data(), s->open_next >= 0 ? s->d_O : s->d_P,
                               sizeof(uint64_t) * (size_t)s->n, hipMemcpyDeviceToHost, st));
    }
    if (elite) {
        E.resize((size_t)((s->n + 63) / 64));
        HIP_TRY(hipMemcpyAsync(E.data(), s->d_E, sizeof(uint64_t) * E.size(),
                               hipMemcpyDeviceToHost, st));
    }
    DevState h;
    int64_t cnt[3];
    int rc = read_fitness_counters(s, st, fit, &h, cnt);
    if (rc) return rc;
    if (genes)
        for (int32_t i = 0; i < s->N; ++i) {
            uint8_t *row = genes + (size_t)i * (size_t)s->n;
            for (int32_t v = 0; v < s->n; ++v) row[v] = (uint8_t)((P[(size_t)v] >> i) & 1u);
        }
    if (elite)
        for (int32_t v = 0; v < s->n; ++v) elite[v] = (uint8_t)((E[(size_t)v >> 6] >> (v & 63)) & 1u);
    if (fitness) std::copy(fit, fit + s->N, fitness);
    if (elite_fitness) *elite_fitness = h.elite_fitness;
    if (generation) *generation = h.generation;
    if (counters) std::copy(cnt, cnt + 3, counters);
    return GOM_OK;
    GUARD_END
}

// Terms of the state hash for `bytes` little-endian bytes of x at positions k, k+1, ...
static uint64_t hash_int(uint64_t &k, uint64_t x, int bytes) {
    uint64_t h = 0;
    for (int t = 0; t < bytes; ++t, ++k) h += mix64((k << 8) | ((x >> (8 * t)) & 0xFFu));
    return h;
}

extern "C" int gom_state_hash(gom_state *s, void *stream, uint64_t *hash) {
    GUARD_BEGIN
    if (!s || !hash) return fail(GOM_E_ARG, "gom_state_hash: null argument");
    hipStream_t st = (hipStream_t)stream;
    const uint64_t n = (uint64_t)s->n, N = (uint64_t)s->N;
    HIP_TRY(launch_state_hash(s->open_next >= 0 ? s->d_O : s->d_P, s->d_E, s->n, s->N,
                              N * n + 8 * N, s->d_st, st));
    int64_t fit[GOM_MAX_POP];
    DevState h;
    int64_t cnt[3];
    int rc = read_fitness_counters(s, st, fit, &h, cnt);
    if (rc) return rc;
    uint64_t acc = h.hash, k = N * n;
    for (int32_t i = 0; i < s->N; ++i) acc += hash_int(k, (uint64_t)fit[i], 8);
    k += n;  // the elitist's bytes, summed on the device
    acc += hash_int(k, (uint64_t)h.elite_fitness, 8);
    acc += hash_int(k, (uint64_t)(uint32_t)h.generation, 4);
    for (int c = 0; c < 3; ++c) acc += hash_int(k, (uint64_t)cnt[c], 8);
    *hash = acc;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_state_write(gom_state *s, void *stream, const uint8_t *genes,
                               const uint8_t *elite, int64_t elite_fitness, int32_t generation,
                               const int64_t *counters) {
    GUARD_BEGIN
    if (!s || !genes || !elite || !counters) return fail(GOM_E_ARG, "gom_state_write: null argument");
    if (generation < 0) return fail(GOM_E_ARG, "gom_state_write: negative generation");
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint64_t> P((size_t)s->n, 0), E((size_t)((s->n + 63) / 64), 0);
    for (int32_t i = 0; i < s->N; ++i) {
        const uint8_t *row = genes + (size_t)i * (size_t)s->n;
        for (int32_t v = 0; v < s->n; ++v) {
            if (row[v] > 1) return fail(GOM_E_ARG, "gom_state_write: gene outside {0, 1}");
            P[(size_t)v] |= (uint64_t)row[v] << i;
        }
    }
    for (int32_t v = 0; v < s->n; ++v) {
        if (elite[v] > 1) return fail(GOM_E_ARG, "gom_state_write: elite gene outside {0, 1}");
        E[(size_t)v >> 6] |= (uint64_t)elite[v] << (v & 63);
    }
    DevState h{};
    h.elite_fitness = elite_fitness;
    h.evaluated = counters[1];
    h.accepted = counters[2];
    h.generation = generation;
    h.done_tick = -1;
    HIP_TRY(hipMemcpyAsync(s->d_P, P.data(), sizeof(uint64_t) * P.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->d_O, P.data(), sizeof(uint64_t) * P.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->d_E, E.data(), sizeof(uint64_t) * E.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->d_st, &h, sizeof(DevState), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_zero_state(s->d_fit, s->d_stripes, st));
    HIP_TRY(launch_full_fitness(s->d_P, s->d_eu, s->d_ev, s->d_ew, s->m, s->N, s->d_stripes, st));
    EpilogueArgs ea{};
    ea.P = s->d_P;
    ea.O = s->d_O;
    ea.E = s->d_E;
    ea.fit = s->d_fit;
    ea.st = s->d_st;
    ea.stripes = s->d_stripes;
    ea.target = INT64_MAX;
    ea.n = s->n;
    ea.N = s->N;
    ea.mode = kEpiRefresh;
    HIP_TRY(launch_epilogue(ea, st));
    HIP_TRY(hipStreamSynchronize(st));
    s->g_host = generation;
    s->g_base = generation;
    s->attempted_base = counters[0];
    s->open_next = -1;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_timing_enable(gom_state *s, int period) {
    if (!s) return fail(GOM_E_ARG, "gom_timing_enable: null state");
    if (period < 0) return fail(GOM_E_ARG, "gom_timing_enable: negative period");
    s->timing = period;
    s->sweep_launches = 0;
    return GOM_OK;
}

extern "C" int gom_timing_read(gom_state *s, double *class_ms_total, int64_t *class_launches) {
    GUARD_BEGIN
    if (!s) return fail(GOM_E_ARG, "gom_timing_read: null state");
    for (size_t q = 0; q + 1 < s->tev_used; q += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(s->tev[q + 1]));
        HIP_TRY(hipEventElapsedTime(&ms, s->tev[q], s->tev[q + 1]));
        s->t_ms += ms;
        s->t_launches++;
    }
    s->tev_used = 0;
    if (class_ms_total) *class_ms_total = s->t_ms;
    if (class_launches) *class_launches = s->t_launches;
    s->t_ms = 0.0;
    s->t_launches = 0;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_state_set_schedule(gom_state *s, int schedule) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_schedule: null state");
    switch (schedule) {
    case GOM_SCHED_AUTO:
        s->sched = auto_schedule(s);
        return GOM_OK;
    case GOM_SCHED_BITSLICED:
        if (!s->bitsliced_ok)
            return fail(GOM_E_RANGE, "gom_state_set_schedule: the bit-sliced schedule needs a "
                        "univariate FOS, maximum degree <= 4 and per-vertex |w| sums < 2^30");
        if (s->fi)
            return fail(GOM_E_RANGE, "gom_state_set_schedule: the bit-sliced schedule has no "
                        "forced improvement");
        s->sched = schedule;
        return GOM_OK;
    case GOM_SCHED_CLASS_LAUNCH:
        s->sched = schedule;
        return GOM_OK;
    case GOM_SCHED_RESIDENT:
        if (!s->resident_ok)
            return fail(GOM_E_RANGE, "gom_state_set_schedule: resident schedule needs %zu bytes "
                        "of LDS and at most %d classes (instance: %d classes)",
                        resident_lds_bytes(s->n, false), kResidentMaxClasses, s->k);
        s->sched = schedule;
        return GOM_OK;
    default:
        return fail(GOM_E_ARG, "gom_state_set_schedule: unknown schedule %d", schedule);
    }
}

extern "C" int gom_state_set_fused(gom_state *s, int enabled) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_fused: null state");
    if (enabled && !s->fused_ok)
        return fail(GOM_E_RANGE, "gom_state_set_fused: the fused bit-sliced sweep does not fit "
                    "this state (needs the bit-sliced schedule's eligibility, at most %d classes "
                    "and dependency ranges of at most %d chunks)", kFusedMaxClasses,
                    kFusedMaxDepChunks);
    s->fused_use = enabled != 0;
    return GOM_OK;
}

extern "C" int gom_state_get_fused(const gom_state *s, int *enabled, int *available) {
    if (!s) return fail(GOM_E_ARG, "gom_state_get_fused: null state");
    if (enabled) *enabled = s->fused_ok && s->fused_use;
    if (available) *available = s->fused_ok;
    return GOM_OK;
}

extern "C" int gom_state_autotune(gom_state *s, int32_t trial_generations, void *stream,
                                  int *chosen) {
    GUARD_BEGIN
    if (!s || trial_generations < 1) return fail(GOM_E_ARG, "gom_state_autotune: bad arguments");
    if (s->open_next >= 0) return fail(GOM_E_STATE, "gom_state_autotune: a generation is open");
    hipStream_t st = (hipStream_t)stream;
    // (schedule, class-launch block size, fused bit-sliced sweep)
    struct Cand {
        int sched, threads;
        bool fused;
    };
    std::vector<Cand> cands;
    for (int t : {64, 128, 256, 512}) cands.push_back({GOM_SCHED_CLASS_LAUNCH, t, s->fused_use});
    if (s->resident_ok) cands.push_back({GOM_SCHED_RESIDENT, s->sweep_threads, s->fused_use});
    if (s->bitsliced_ok && !s->fi) {
        cands.push_back({GOM_SCHED_BITSLICED, s->sweep_threads, false});
        if (s->fused_ok) cands.push_back({GOM_SCHED_BITSLICED, s->sweep_threads, true});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GOM_E_DEVICE, "gom_state_autotune: %s", hipGetErrorString(he));
    }
    const bool timing = s->timing != 0;
    s->timing = 0;
    // two interleaved rounds; each candidate keeps its faster round
    constexpr int kRounds = 2;
    std::vector<float> cand_ms(cands.size(), 0.f);
    int rc = GOM_OK;
    for (int round = 0; round < kRounds && rc == GOM_OK; ++round) {
        for (size_t ci = 0; ci < cands.size() && rc == GOM_OK; ++ci) {
            s->sched = cands[ci].sched;
            s->sweep_threads = cands[ci].threads;
            s->fused_use = cands[ci].fused;
            // one untimed generation loads the schedule's kernels, then the timed ones
            for (int32_t t = 0; t <= trial_generations && rc == GOM_OK; ++t) {
                if (t == 1 && hipEventRecord(e0, st) != hipSuccess) rc = GOM_E_DEVICE;
                if (rc == GOM_OK) rc = enqueue_generation(s, s->g_host, INT64_MAX, st);
                if (rc == GOM_OK) s->g_host++;
            }
            if (rc == GOM_OK && hipEventRecord(e1, st) != hipSuccess) rc = GOM_E_DEVICE;
            float ms = 0.f;
            if (rc == GOM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = GOM_E_DEVICE;
            if (rc == GOM_OK && (round == 0 || ms < cand_ms[ci])) cand_ms[ci] = ms;
        }
    }
    Cand best = cands.front();
    float best_ms = cand_ms.front();
    for (size_t ci = 1; ci < cands.size(); ++ci)
        if (cand_ms[ci] < best_ms) {
            best_ms = cand_ms[ci];
            best = cands[ci];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->timing = timing;
    if (rc != GOM_OK) return fail(rc, "gom_state_autotune: a trial generation failed");
    s->sched = best.sched;
    s->sweep_threads = best.threads;
    s->fused_use = best.fused;
    if (chosen) *chosen = best.sched;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_state_set_block(gom_state *s, int threads) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_block: null state");
    if (threads < 64 || threads > 512 || threads % 64)
        return fail(GOM_E_RANGE, "gom_state_set_block: %d threads (64..512, a multiple of 64)",
                    threads);
    s->sweep_threads = threads;
    return GOM_OK;
}

extern "C" int gom_state_set_staged(gom_state *s, int enabled) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_staged: null state");
    s->staged_use = enabled != 0;
    return GOM_OK;
}

extern "C" int gom_state_set_grid_limit(gom_state *s, int32_t blocks) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_grid_limit: null state");
    if (blocks < 1 || blocks > 65536)
        return fail(GOM_E_RANGE, "gom_state_set_grid_limit: %d blocks (1..65536)", blocks);
    s->max_grid = blocks;
    s->swar_narrow = s->swar_uni && swar_narrow_ok(s);
    return GOM_OK;
}

extern "C" int gom_state_set_bitsliced_min_sets(gom_state *s, int32_t sets) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_bitsliced_min_sets: null state");
    if (sets < 0) return fail(GOM_E_RANGE, "gom_state_set_bitsliced_min_sets: %d sets", sets);
    s->gs_min_sets = sets;
    s->bitsliced_ok = s->swar_uni || gs_select(s);
    if (s->sched == GOM_SCHED_BITSLICED && !s->bitsliced_ok) s->sched = auto_schedule(s);
    return GOM_OK;
}

extern "C" int gom_state_get_block(const gom_state *s, int *threads) {
    if (!s || !threads) return fail(GOM_E_ARG, "gom_state_get_block: null argument");
    *threads = s->sweep_threads;
    return GOM_OK;
}

extern "C" int gom_state_set_fi(gom_state *s, int enabled) {
    if (!s) return fail(GOM_E_ARG, "gom_state_set_fi: null state");
    if (s->open_next >= 0) return fail(GOM_E_STATE, "gom_state_set_fi: a generation is open");
    s->fi = enabled != 0;
    if (s->fi && s->sched == GOM_SCHED_BITSLICED) s->sched = auto_schedule(s);
    return GOM_OK;
}

extern "C" int gom_state_get_fi(const gom_state *s, int *enabled) {
    if (!s || !enabled) return fail(GOM_E_ARG, "gom_state_get_fi: null argument");
    *enabled = s->fi ? 1 : 0;
    return GOM_OK;
}

extern "C" int gom_state_get_schedule(const gom_state *s, int *schedule) {
    if (!s || !schedule) return fail(GOM_E_ARG, "gom_state_get_schedule: null argument");
    *schedule = s->sched;
    return GOM_OK;
}

extern "C" int gom_state_info(const gom_state *s, int32_t *n, int32_t *pop, int32_t *n_sets,
                              int32_t *n_classes, int32_t *max_class) {
    if (!s) return fail(GOM_E_ARG, "gom_state_info: null state");
    if (n) *n = s->n;
    if (pop) *pop = s->N;
    if (n_sets) *n_sets = s->n_sets;
    if (n_classes) *n_classes = s->k;
    if (max_class) *max_class = s->max_class;
    return GOM_OK;
}

extern "C" void gom_state_free(gom_state *s) {
    if (!s) return;
    for (hipEvent_t e : s->tev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->chunk_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->h_st) {
        if (s->h_st_pinned) (void)hipHostFree(s->h_st);
        else delete[] s->h_st;
    }
    if (s->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[(size_t)s->static_dev] = false;
    }
    delete s;
}

// ------------------------------------------------------------------------------------------
// Batches of independent instances
// ------------------------------------------------------------------------------------------
struct gom_batch {
    int32_t count = 0;
    std::vector<gom_state *> subs;      // owned
    std::vector<int64_t> targets;
    BatchInst *d_insts = nullptr;
    int2 *d_blk = nullptr;
    int32_t *d_vblk = nullptr;
    DevState *d_snap = nullptr;         // packed copy of the instances' run scalars
    int vblocks = 0;
    std::vector<BatchLaunch> groups;    // sweep launch groups of the current block sizes
    std::vector<int32_t> solo;          // instances that run their own sweeps in each step
    std::vector<int32_t> bcl;           // instances swept by the batched class launches
    int64_t bcl_min_n = -1;             // ... those eligible with at least this many vertices
    BclInst *d_bcl = nullptr;
    uint16_t *d_bcl_order = nullptr;
    int32_t *d_bcl_tiles = nullptr;
    int bcl_kmax = 0, bcl_grid = 0;
    int bcl_ppw = 2;                    // class positions per wave of the class launches
    uint64_t *d_bcl_nzm = nullptr;      // per class-launched instance: neutral-step mask
    int4 *d_bcl_pos = nullptr;          // per position and instance: its class (bit-sliced form)
    bool bcl_gs_use = true;             // class launches in the bit-sliced form when ...
    bool bcl_gs_ok = false;             // ... every class-launched instance admits it
    int bcl_gs_wb = 0, bcl_gs_grid = 0; // its weight bits (7 or 13) and blocks per launch
    int64_t narrow_max_n = -1;          // instances with n <= this run 256-thread blocks
    size_t lds_max = 0;                 // LDS per CU of the device
    DevState *h_st = nullptr;           // pinned, 2 x count
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};
    double wall_khz = 0.0;
    int32_t g_done = 0;                 // generation steps run
    bool use_graph = true;              // chunks of kBatchChunk steps as a captured graph
    hipStream_t cap = nullptr;          // private stream the graph is captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<BatchInst> h_insts;     // host copy of the instance table
    bool timing = false;                // every sweep launch records a pair of events
    std::vector<hipEvent_t> tev;        // event pool of the timed sweep launches
    size_t tev_used = 0;
    double t_ms = 0.0;                  // folded sweep time and launch count
    int64_t t_launches = 0;
};

namespace {
struct BatchLayout {
    std::vector<size_t> sub_off, sub_bytes;
    size_t insts = 0, blk = 0, vblk = 0, snap = 0, bcl = 0, bcl_order = 0, bcl_tiles = 0,
           bcl_nzm = 0, bcl_pos = 0, total = 0;
    int sweep_blocks = 0, vblocks = 0, kmax = 0;
};

int batch_layout(int32_t count, const mc_graph *const *graphs, const gom_fos *const *fos,
                 const int32_t *pops, BatchLayout &B) {
    size_t o = 0;
    B.sub_off.resize((size_t)count);
    B.sub_bytes.resize((size_t)count);
    int sweep = 0, vb = 0;
    for (int32_t b = 0; b < count; ++b) {
        size_t bytes = 0;
        int rc = gom_state_bytes(graphs[b], fos[b], pops[b], &bytes);
        if (rc) return rc;
        B.sub_off[(size_t)b] = o;
        B.sub_bytes[(size_t)b] = bytes;
        o = align_up(o + bytes);
        sweep += pops[b];
        vb += (graphs[b]->n + 255) / 256;
    }
    B.insts = o;
    o = align_up(o + sizeof(BatchInst) * (size_t)count);
    B.blk = o;
    o = align_up(o + sizeof(int2) * (size_t)sweep);
    B.vblk = o;
    o = align_up(o + sizeof(int32_t) * (size_t)vb);
    B.snap = o;
    o = align_up(o + sizeof(DevState) * (size_t)count);
    // batched class launches: room for every instance (which ones take them is decided later)
    int kmax = 1;
    for (int32_t b = 0; b < count; ++b) kmax = std::max(kmax, fos[b]->k);
    B.bcl = o;
    o = align_up(o + sizeof(BclInst) * (size_t)count);
    B.bcl_order = o;
    o = align_up(o + sizeof(uint16_t) * (size_t)count * kmax);
    B.bcl_tiles = o;
    o = align_up(o + sizeof(int32_t) * (size_t)kmax * (count + 1));
    B.bcl_nzm = o;
    o = align_up(o + sizeof(uint64_t) * (size_t)count);
    B.bcl_pos = o;
    o = align_up(o + 2 * sizeof(int4) * (size_t)kmax * count);
    B.total = o;
    B.sweep_blocks = sweep;
    B.vblocks = vb;
    B.kmax = kmax;
    return GOM_OK;
}
}  // namespace

extern "C" int gom_batch_bytes(int32_t count, const mc_graph *const *graphs,
                               const gom_fos *const *fos, const int32_t *pops, size_t *bytes) {
    GUARD_BEGIN
    if (count < 1 || !graphs || !fos || !pops || !bytes)
        return fail(GOM_E_ARG, "gom_batch_bytes: bad arguments");
    BatchLayout B;
    int rc = batch_layout(count, graphs, fos, pops, B);
    if (rc) return rc;
    *bytes = B.total;
    return GOM_OK;
    GUARD_END
}

extern "C" void gom_batch_free(gom_batch *b) {
    if (!b) return;
    for (gom_state *s : b->subs) gom_state_free(s);
    for (hipEvent_t e : b->chunk_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->tev) (void)hipEventDestroy(e);
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->h_st) (void)hipHostFree(b->h_st);
    delete b;
}

// Default block-size threshold of the batched sweep: instances with at most this many vertices
// run 256-thread blocks, larger ones 1024.
constexpr int64_t kBatchNarrowDefault = 16384;
// Default vertex count from which eligible instances take the batched class launches.
constexpr int64_t kBatchClassMinDefault = 20000;

// Sweep blocks of one CU that the LDS of a block allows (at most 8).
static int blocks_per_cu(size_t lds, size_t lds_max) {
    return (int)std::min<size_t>(8, lds ? lds_max / lds : 8);
}

// Blocks per CU by registers and threads of each (threads, kind) variant of the batched sweep,
// looked up once per process (the library's device code is the same on every device).
static int batch_reg_blocks(int threads, int kind) {
    static std::mutex mu;
    static int cache[2][2] = {{0, 0}, {0, 0}};
    std::lock_guard<std::mutex> lk(mu);
    int &c = cache[threads == 256 ? 0 : 1][kind ? 1 : 0];
    if (c == 0) {
        int b = 0;
        if (batch_sweep_occupancy(threads, kind, &b) != hipSuccess || b < 1) b = 1;
        c = b;
    }
    return c;
}

// Block sizes, P copies and launch groups for the threshold `narrow_max_n`: an instance with
// n <= narrow_max_n sweeps with 256-thread blocks, else 1024.  It keeps a copy of P in LDS
// when that does not lower the blocks a CU can hold.  Instances with equal (threads, blocks
// per CU) form one launch; within it, instances with more classes and vertices per thread
// (longer blocks) come first.  Uploads the instance table and the block map (synchronous)
// and drops a captured graph.
// May instance s take the batched class launches (general records of sets of at most
// kBclMaxMembers members and kBclMaxEntries dependent edges)?
static bool bcl_eligible(const gom_state *s) {
    if (s->univariate || s->max_set > kBclMaxMembers || s->k > 2048) return false;
    for (int32_t e : s->class_entries)
        if (e > kBclMaxEntries) return false;
    return true;
}

// Drop the captured chunk graph (it holds the launch arguments of the current plan).
static void drop_graph(gom_batch *b) {
    if (b->graph_exec) {
        (void)hipGraphExecDestroy(b->graph_exec);
        b->graph_exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
}

// May general instance s take the bit-sliced form of the class launches (population <= 64,
// per-set |w| sums and |w| within the bounds of the bit-sliced sum)?
static bool gs_admissible(const gom_state *s) {
    if (s->N > 64) return false;
    for (int32_t c = 0; c < s->k; ++c) {
        int bits = 1;
        while (bits < 62 && (s->class_wmax[c] >> bits) != 0) ++bits;
        if (s->class_wsum[c] > kGsMaxWeightSum || bits > kGsMaxWeightBits) return false;
    }
    return true;
}

static int batch_regroup(gom_batch *b, int64_t narrow_max_n, int64_t bcl_min_n,
                         hipStream_t st) {
    // which instances the batched class launches sweep (the others: resident blocks)
    std::vector<BclInst> bi;
    b->bcl.clear();
    b->bcl_kmax = 0;
    // the bit-sliced form is admitted when every general instance that takes the class
    // launches admits it; univariate instances that the univariate bit-sliced sweep fits then
    // take the class launches as well, one lane a set (the lane-per-solution form reads only
    // general records)
    bool gs_ok = true, any = false;
    for (int32_t i = 0; i < b->count; ++i) {
        const gom_state *s = b->subs[(size_t)i];
        if (b->h_insts[(size_t)i].solo || bcl_min_n < 0 || (int64_t)s->n < bcl_min_n ||
            !bcl_eligible(s))
            continue;
        any = true;
        if (!gs_admissible(s)) gs_ok = false;
    }
    const bool gs = gs_ok && b->bcl_gs_use;
    for (int32_t i = 0; i < b->count; ++i) {
        BatchInst &I = b->h_insts[(size_t)i];
        const gom_state *s = b->subs[(size_t)i];
        if (I.solo) continue;
        const bool uni = gs && s->univariate && s->swar_uni && s->N <= 64;
        I.bcl = bcl_min_n >= 0 && (int64_t)s->n >= bcl_min_n && (bcl_eligible(s) || uni);
        any |= I.bcl;
        I.epi = epilogue_args(s, b->targets[(size_t)i], !I.bcl);
        if (!I.bcl) continue;
        BclInst c{};
        c.P = s->d_P;
        c.O = s->d_O;
        c.stripes = s->d_stripes;
        c.st = s->d_st;
        c.roff = s->d_roff;
        c.recs = s->d_recs;
        c.class_ptr = s->d_cptr;
        c.class_rec = s->d_crec;
        c.seed = s->seed;
        c.target = b->targets[(size_t)i];
        c.N = s->N;
        c.always = s->rule == GOM_NEUTRAL_ALWAYS;
        c.k = s->k;
        c.order_fixed = s->order == GOM_ORDER_FIXED;
        c.uni = s->univariate ? 1 : 0;
        c.sw = s->d_sw;
        c.sw_stride = s->sw_stride;
        c.partition = s->partition ? 1 : 0;
        bi.push_back(c);
        b->bcl.push_back(i);
        b->bcl_kmax = std::max(b->bcl_kmax, s->k);
    }
    if (!bi.empty() && b->bcl_grid == 0) HIP_TRY(bcl_sweep_grid(&b->bcl_grid));
    // the bit-sliced form's launch grid: the most slots a position can have (every instance
    // at its largest class), and its weight bits (the general instances')
    b->bcl_gs_ok = any && gs_ok;
    int wbits = 1;
    int64_t slots = 0;
    for (int32_t i : b->bcl) {
        const gom_state *s = b->subs[(size_t)i];
        if (s->univariate) {
            slots += gs_slots_uni(s->max_class);
            continue;
        }
        for (int32_t c = 0; c < s->k; ++c) {
            int bits = 1;
            while (bits < 62 && (s->class_wmax[c] >> bits) != 0) ++bits;
            wbits = std::max(wbits, bits);
        }
        slots += gs_slots_bcl(s->max_class, s->N > 32 ? 2 : 1);
    }
    b->bcl_gs_wb = wbits <= 7 ? 7 : 13;
    b->bcl_gs_grid = (int)std::min<int64_t>((slots + kGsThreads - 1) / kGsThreads, 1 << 30);
    struct Item {
        int threads, kind, occ;
        double cost;
        int32_t inst;
        size_t lds;
    };
    std::vector<Item> items;
    items.reserve((size_t)b->count);
    for (int32_t i = 0; i < b->count; ++i) {
        const gom_state *s = b->subs[(size_t)i];
        if (b->h_insts[(size_t)i].solo || b->h_insts[(size_t)i].bcl) continue;
        int T = (int64_t)s->n <= narrow_max_n ? 256 : 1024;
        if (kBatchOrderBytes + resident_lds_bytes(s->n, false, T) > b->lds_max) T = 256;
        const size_t l0 = kBatchOrderBytes + resident_lds_bytes(s->n, false, T);
        const size_t l1 = kBatchOrderBytes + resident_lds_bytes(s->n, true, T);
        if (l0 > b->lds_max)
            return fail(GOM_E_RANGE, "batch: instance %d needs %zu bytes of LDS", i, l0);
        const int kind = s->univariate ? 0 : 1;
        const int reg = batch_reg_blocks(T, kind);
        const bool plds = l1 <= b->lds_max && std::min(blocks_per_cu(l1, b->lds_max), reg) ==
                                                  std::min(blocks_per_cu(l0, b->lds_max), reg);
        b->h_insts[(size_t)i].plds = plds ? 1 : 0;
        const size_t l = plds ? l1 : l0;
        const double cost = (double)s->k + (double)s->n_sets / T;
        const int occ = std::min(blocks_per_cu(l, b->lds_max), reg);
        items.push_back(Item{T, kind, occ, cost, i, l});
    }
    std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) {
        if (x.threads != y.threads) return x.threads > y.threads;
        if (x.kind != y.kind) return x.kind > y.kind;
        if (x.occ != y.occ) return x.occ < y.occ;
        return x.cost > y.cost;
    });
    // Launch groups; inside a group, every instance's blocks go to one XCD (the dispatcher
    // sends block j of a launch to XCD j mod 8): instances are spread over the 8 XCDs by
    // decreasing work (population x block cost) onto the least loaded, and the block list
    // interleaves the XCDs' lists, so an instance's records and population words are fetched
    // into one L2 instead of eight.  A list that runs out early is topped up from the longest.
    std::vector<int2> blk;
    std::vector<BatchLaunch> groups;
    constexpr int kXcds = 8;
    size_t q0 = 0;
    while (q0 < items.size()) {
        size_t q1 = q0 + 1;
        while (q1 < items.size() && items[q1].threads == items[q0].threads &&
               items[q1].kind == items[q0].kind && items[q1].occ == items[q0].occ)
            ++q1;
        BatchLaunch G{(int)blk.size(), 0, items[q0].threads, items[q0].kind, 0};
        std::vector<std::deque<int2>> bins(kXcds);
        std::vector<double> load(kXcds, 0.0);
        std::vector<size_t> order;
        for (size_t q = q0; q < q1; ++q) order.push_back(q);
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            const double wx = items[x].cost * b->subs[(size_t)items[x].inst]->N;
            const double wy = items[y].cost * b->subs[(size_t)items[y].inst]->N;
            return wx > wy;
        });
        for (size_t q : order) {
            const Item &it = items[q];
            const int32_t N = b->subs[(size_t)it.inst]->N;
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[(size_t)x] += it.cost * N;
            for (int32_t i = 0; i < N; ++i) bins[(size_t)x].push_back(make_int2(it.inst, i));
            G.count += N;
            G.lds = std::max(G.lds, it.lds);
        }
        // each XCD's list longest blocks first (the instances were placed in that order of
        // work, and a block's cost decides its length)
        for (auto &bin : bins)
            std::stable_sort(bin.begin(), bin.end(), [&](const int2 &u, const int2 &v) {
                auto cost = [&](const int2 &e) {
                    const gom_state *s = b->subs[(size_t)e.x];
                    return (double)s->k + (double)s->n_sets / G.threads;
                };
                return cost(u) > cost(v);
            });
        for (int j = 0; j < G.count; ++j) {
            size_t x = (size_t)(j % kXcds);
            if (bins[x].empty()) {
                size_t best = 0;
                for (size_t y = 1; y < bins.size(); ++y)
                    if (bins[y].size() > bins[best].size()) best = y;
                x = best;
            }
            blk.push_back(bins[x].front());
            bins[x].pop_front();
        }
        groups.push_back(G);
        q0 = q1;
    }
    HIP_TRY(hipStreamSynchronize(st));  // nothing in flight reads the tables
    HIP_TRY(hipMemcpyAsync(b->d_insts, b->h_insts.data(), sizeof(BatchInst) * b->h_insts.size(),
                           hipMemcpyHostToDevice, st));
    if (!blk.empty())
        HIP_TRY(hipMemcpyAsync(b->d_blk, blk.data(), sizeof(int2) * blk.size(),
                               hipMemcpyHostToDevice, st));
    if (!bi.empty())
        HIP_TRY(hipMemcpyAsync(b->d_bcl, bi.data(), sizeof(BclInst) * bi.size(),
                               hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(prepare_batch_step(groups.data(), (int)groups.size()));
    drop_graph(b);
    b->groups = std::move(groups);
    b->narrow_max_n = narrow_max_n;
    b->bcl_min_n = bcl_min_n;
    return GOM_OK;
}

// The batched class launches' plan arguments of the batch's current assignment.
static BclPlan bcl_plan(const gom_batch *b) {
    BclPlan p{};
    p.insts = b->d_bcl;
    p.order = b->d_bcl_order;
    p.tiles = b->d_bcl_tiles;
    p.count = (int32_t)b->bcl.size();
    p.kmax = b->bcl_kmax;
    p.grid = b->bcl_grid;
    p.ppw = b->bcl_ppw;
    p.gs = b->bcl_gs_ok && b->bcl_gs_use ? 1 : 0;
    p.gs_wb = b->bcl_gs_wb;
    p.gs_grid = b->bcl_gs_grid;
    p.nzm = b->d_bcl_nzm;
    p.pos = b->d_bcl_pos;
    return p;
}

extern "C" int gom_batch_init(int32_t count, const mc_graph *const *graphs,
                              const gom_fos *const *fos, const int32_t *pops,
                              const uint64_t *seeds, const int64_t *targets, int neutral_rule,
                              int class_order, void *dev_arena, size_t arena_bytes,
                              void *stream, gom_batch **out) {
    GUARD_BEGIN
    if (count < 1 || !graphs || !fos || !pops || !seeds || !targets || !dev_arena || !out)
        return fail(GOM_E_ARG, "gom_batch_init: bad arguments");
    BatchLayout B;
    int rc = batch_layout(count, graphs, fos, pops, B);
    if (rc) return rc;
    if (arena_bytes < B.total)
        return fail(GOM_E_NOMEM, "gom_batch_init: arena has %zu bytes, needs %zu", arena_bytes,
                    B.total);
    if ((reinterpret_cast<uintptr_t>(dev_arena) & 255) != 0)
        return fail(GOM_E_NOMEM, "gom_batch_init: arena must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char *arena = (char *)dev_arena;
    auto *bt = new gom_batch;
    bt->count = count;
    bt->targets.assign(targets, targets + count);
    auto cleanup = [&](int code) {
        gom_batch_free(bt);
        return code;
    };
    std::vector<BatchInst> insts((size_t)count);
    std::vector<int2> blk;
    std::vector<int32_t> vblk;
    for (int32_t b = 0; b < count; ++b) {
        gom_state *s = nullptr;
        rc = gom_state_init(graphs[b], fos[b], pops[b], seeds[b], neutral_rule, class_order,
                            arena + B.sub_off[(size_t)b], B.sub_bytes[(size_t)b], stream, &s);
        if (rc) return cleanup(rc);
        bt->subs.push_back(s);
        const size_t need = kBatchOrderBytes + resident_lds_bytes(s->n, false, 256);
        bt->lds_max = s->lds_max;
        BatchInst &I = insts[(size_t)b];
        I.plds = 0;  // set with the block sizes (batch_regroup)
        I.res = resident_ctx(s, targets[b]);
        I.kind = s->univariate ? 0 : 1;
        I.order_fixed = s->order == GOM_ORDER_FIXED;
        // an instance beyond the resident schedule (LDS or classes) runs its own sweeps in
        // each step, with the schedule its state chose (bit-sliced or class launch)
        I.solo = !s->resident_ok || need > s->lds_max;
        I.epi = epilogue_args(s, targets[b], !I.solo);
        I.vblock0 = (int32_t)vblk.size();
        if (I.solo) {
            if (s->sched == GOM_SCHED_RESIDENT) s->sched = GOM_SCHED_CLASS_LAUNCH;
            bt->solo.push_back(b);
        } else {
            for (int32_t q = 0; q < (s->n + 255) / 256; ++q) vblk.push_back(b);
        }
    }
    bt->d_bcl = (BclInst *)(arena + B.bcl);
    bt->d_bcl_order = (uint16_t *)(arena + B.bcl_order);
    bt->d_bcl_tiles = (int32_t *)(arena + B.bcl_tiles);
    bt->d_bcl_nzm = (uint64_t *)(arena + B.bcl_nzm);
    bt->d_bcl_pos = (int4 *)(arena + B.bcl_pos);
    bt->d_insts = (BatchInst *)(arena + B.insts);
    bt->d_blk = (int2 *)(arena + B.blk);
    bt->d_vblk = (int32_t *)(arena + B.vblk);
    bt->d_snap = (DevState *)(arena + B.snap);
    bt->vblocks = (int)vblk.size();
    int khz = 0, dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_insts, insts.data(), sizeof(BatchInst) * insts.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_vblk, vblk.data(), sizeof(int32_t) * vblk.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&bt->h_st, 2 * sizeof(DevState) * (size_t)count,
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->chunk_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->chunk_ev[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return cleanup(fail(GOM_E_DEVICE, "gom_batch_init: %s", hipGetErrorString(e)));
    bt->wall_khz = (double)khz;
    bt->h_insts = std::move(insts);
    rc = batch_regroup(bt, kBatchNarrowDefault, kBatchClassMinDefault, st);
    if (rc) return cleanup(rc);
    *out = bt;
    return GOM_OK;
    GUARD_END
}

// Copy every instance's run scalars into pinned slot `slot` (asynchronous): a gather kernel
// packs them next to each other, then one copy.
static hipError_t batch_snapshot(gom_batch *b, int slot, hipStream_t st) {
    DevState *dst = b->h_st + (size_t)slot * (size_t)b->count;
    hipError_t e = launch_batch_gather(b->d_insts, b->count, b->d_snap, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(dst, b->d_snap, sizeof(DevState) * (size_t)b->count,
                          hipMemcpyDeviceToHost, st);
}

// One chunk of generation steps and the gather of the run scalars, captured once as a graph.
static hipError_t batch_chunk_graph(gom_batch *b, int32_t steps) {
    if (b->graph_exec) return hipSuccess;
    hipError_t e = prepare_batch_step(b->groups.data(), (int)b->groups.size());
    if (e == hipSuccess && !b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int32_t t = 0; t < steps && le == hipSuccess; ++t)
        le = launch_batch_step(b->d_insts, b->count, b->d_blk, b->groups.data(),
                               (int)b->groups.size(), b->d_vblk, b->vblocks, bcl_plan(b),
                               b->cap);
    if (le == hipSuccess) le = launch_batch_gather(b->d_insts, b->count, b->d_snap, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);  // always ends the capture
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    b->graph = g;
    b->graph_exec = x;
    return hipSuccess;
}

static bool batch_all_done(const gom_batch *b, int slot) {
    const DevState *h = b->h_st + (size_t)slot * (size_t)b->count;
    for (int32_t i = 0; i < b->count; ++i)
        if (h[i].elite_fitness < b->targets[(size_t)i]) return false;
    return true;
}

// `steps` generations of every instance that runs its own sweeps (solo), enqueued after the
// batched launches of the same steps; its generation index is kept on the host.
static int batch_solo_steps(gom_batch *b, int32_t steps, hipStream_t st) {
    for (int32_t i : b->solo) {
        gom_state *s = b->subs[(size_t)i];
        for (int32_t t = 0; t < steps; ++t) {
            const int rc = enqueue_generation(s, s->g_host, b->targets[(size_t)i], st);
            if (rc) return rc;
            s->g_host++;
        }
    }
    return GOM_OK;
}

// Events of the next timed sweep launch (timing on), from the batch's pool; when the pool is
// full, the recorded pairs are folded into the running total first.
static int batch_timing_events(gom_batch *b, KernelEvents *ev) {
    *ev = KernelEvents{};
    if (!b->timing) return GOM_OK;
    if (b->tev_used + 2 > b->tev.size()) {
        if (b->tev.size() < (size_t)(1 << 12)) {
            const size_t grow = b->tev.size() ? b->tev.size() : 64;
            for (size_t q = 0; q < grow; ++q) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                b->tev.push_back(e);
            }
        } else {
            for (size_t q = 0; q + 1 < b->tev_used; q += 2) {
                float ms = 0.f;
                HIP_TRY(hipEventSynchronize(b->tev[q + 1]));
                HIP_TRY(hipEventElapsedTime(&ms, b->tev[q], b->tev[q + 1]));
                b->t_ms += ms;
                b->t_launches++;
            }
            b->tev_used = 0;
        }
    }
    ev->start = b->tev[b->tev_used++];
    ev->stop = b->tev[b->tev_used++];
    return GOM_OK;
}

extern "C" int gom_batch_timing_enable(gom_batch *b, int enabled) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_timing_enable: null batch");
    b->timing = enabled != 0;
    return GOM_OK;
}

extern "C" int gom_batch_timing_read(gom_batch *b, double *sweep_ms_total,
                                     int64_t *sweep_launches) {
    GUARD_BEGIN
    if (!b) return fail(GOM_E_ARG, "gom_batch_timing_read: null batch");
    for (size_t q = 0; q + 1 < b->tev_used; q += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(b->tev[q + 1]));
        HIP_TRY(hipEventElapsedTime(&ms, b->tev[q], b->tev[q + 1]));
        b->t_ms += ms;
        b->t_launches++;
    }
    b->tev_used = 0;
    if (sweep_ms_total) *sweep_ms_total = b->t_ms;
    if (sweep_launches) *sweep_launches = b->t_launches;
    b->t_ms = 0.0;
    b->t_launches = 0;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_batch_reseed(gom_batch *b, const uint64_t *seeds, void *stream) {
    GUARD_BEGIN
    if (!b || !seeds) return fail(GOM_E_ARG, "gom_batch_reseed: bad arguments");
    for (int32_t i = 0; i < b->count; ++i)
        if (b->subs[(size_t)i]->open_next >= 0)
            return fail(GOM_E_STATE, "gom_batch_reseed: instance %d has an open generation", i);
    hipStream_t st = (hipStream_t)stream;
    // the previous upload of the table may still read it: wait before rewriting it
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t i = 0; i < b->count; ++i) {
        gom_state *s = b->subs[(size_t)i];
        s->seed = seeds[i];
        HIP_TRY(enqueue_initial_population(s, st));
        b->h_insts[(size_t)i].res.seed = seeds[i];
    }
    // the instance tables carry the seeds (the class launches' table too): upload them again
    const int rc = batch_regroup(b, b->narrow_max_n, b->bcl_min_n, st);
    if (rc) return rc;
    b->g_done = 0;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_batch_run(gom_batch *b, int32_t max_generations, void *stream,
                             gom_result *results, double *time_to_target_ms) {
    GUARD_BEGIN
    if (!b) return fail(GOM_E_ARG, "gom_batch_run: null batch");
    for (int32_t i = 0; i < b->count; ++i)
        if (b->subs[(size_t)i]->open_next >= 0)
            return fail(GOM_E_STATE, "gom_batch_run: instance %d has an open generation", i);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_batch_mark(b->d_insts, b->count, st));
    HIP_TRY(batch_snapshot(b, 0, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<int32_t> g0((size_t)b->count);
    for (int32_t i = 0; i < b->count; ++i) {
        g0[(size_t)i] = b->h_st[i].generation;
        b->subs[(size_t)i]->g_host = b->h_st[i].generation;
    }
    constexpr int32_t kChunk = 4;
    if (!batch_all_done(b, 0)) {
        int32_t issued = b->g_done;
        int slot = 0, prev = -1;
        for (;;) {
            const int32_t n = std::min(kChunk, max_generations - issued);
            int cur = -1;
            if (n > 0) {
                cur = slot;
                if (n == kChunk && b->use_graph && !b->timing) {
                    HIP_TRY(batch_chunk_graph(b, kChunk));
                    HIP_TRY(hipGraphLaunch(b->graph_exec, st));
                    if (!b->solo.empty()) {
                        // the solo instances' generations (their class orders are drawn on
                        // the host, so they stay out of the graph), then the scalars again
                        const int rc = batch_solo_steps(b, kChunk, st);
                        if (rc) return rc;
                        HIP_TRY(launch_batch_gather(b->d_insts, b->count, b->d_snap, st));
                    }
                    HIP_TRY(hipMemcpyAsync(b->h_st + (size_t)cur * (size_t)b->count, b->d_snap,
                                           sizeof(DevState) * (size_t)b->count,
                                           hipMemcpyDeviceToHost, st));
                } else {
                    for (int32_t t = 0; t < n; ++t) {
                        KernelEvents ev;
                        // (a step of solo instances only has no batched sweep to time)
                        const int rc = b->groups.empty() && b->bcl.empty()
                                           ? GOM_OK
                                           : batch_timing_events(b, &ev);
                        if (rc) return rc;
                        HIP_TRY(launch_batch_step(b->d_insts, b->count, b->d_blk,
                                                  b->groups.data(), (int)b->groups.size(),
                                                  b->d_vblk, b->vblocks, bcl_plan(b), st,
                                                  ev));
                        const int src = batch_solo_steps(b, 1, st);
                        if (src) return src;
                    }
                    HIP_TRY(batch_snapshot(b, cur, st));
                }
                issued += n;
                HIP_TRY(hipEventRecord(b->chunk_ev[cur], st));
                slot ^= 1;
            }
            if (prev >= 0) {
                HIP_TRY(hipEventSynchronize(b->chunk_ev[prev]));
                if (batch_all_done(b, prev)) break;
            }
            if (cur < 0) break;
            prev = cur;
        }
        b->g_done = issued;
    }
    HIP_TRY(batch_snapshot(b, 0, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t i = 0; i < b->count; ++i) {
        const DevState &h = b->h_st[i];
        gom_state *s = b->subs[(size_t)i];
        s->g_host = h.generation;
        if (results) {
            gom_result &r = results[i];
            r.generations = h.generation - g0[(size_t)i];
            r.reached = h.elite_fitness >= b->targets[(size_t)i];
            r.best = h.elite_fitness;
            r.attempted = s->attempted_base +
                          (int64_t)s->N * s->n_sets * (int64_t)(h.generation - s->g_base);
            r.evaluated = h.evaluated;
            r.accepted = h.accepted;
        }
        if (time_to_target_ms)
            time_to_target_ms[i] = h.done_tick >= 0 && b->wall_khz > 0
                                       ? (double)(h.done_tick - h.start_tick) / b->wall_khz
                                       : -1.0;
    }
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_batch_set_graph(gom_batch *b, int enabled) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_set_graph: null batch");
    b->use_graph = enabled != 0;
    return GOM_OK;
}

extern "C" int gom_batch_set_narrow(gom_batch *b, int64_t narrow_max_n, void *stream) {
    GUARD_BEGIN
    if (!b) return fail(GOM_E_ARG, "gom_batch_set_narrow: null batch");
    return batch_regroup(b, narrow_max_n, b->bcl_min_n, (hipStream_t)stream);
    GUARD_END
}

extern "C" int gom_batch_get_narrow(const gom_batch *b, int64_t *narrow_max_n,
                                    int32_t *launches) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_get_narrow: null batch");
    if (narrow_max_n) *narrow_max_n = b->narrow_max_n;
    if (launches) *launches = (int32_t)b->groups.size();
    return GOM_OK;
}

// Thresholds from `list` that give distinct assignments of the instances' sizes (the number
// of instances with n <= threshold, or with n >= threshold when `at_least`).
static std::vector<int64_t> distinct_thresholds(const gom_batch *b, std::vector<int64_t> list,
                                                bool at_least) {
    std::vector<int64_t> sizes;
    for (const gom_state *s : b->subs) sizes.push_back(s->n);
    std::sort(sizes.begin(), sizes.end());
    auto key = [&](int64_t c) {
        if (at_least) {
            if (c < 0) return (size_t)0;  // (a negative class-launch threshold: none)
            return (size_t)(sizes.end() - std::lower_bound(sizes.begin(), sizes.end(), c));
        }
        return (size_t)(std::upper_bound(sizes.begin(), sizes.end(), c) - sizes.begin());
    };
    std::vector<int64_t> out;
    for (int64_t c : list) {
        bool dup = false;
        for (int64_t d : out) dup |= key(d) == key(c);
        if (!dup) out.push_back(c);
    }
    return out;
}

extern "C" int gom_batch_autotune(gom_batch *b, int32_t trial_steps, void *stream,
                                  int64_t *narrow_out, int64_t *class_min_out) {
    GUARD_BEGIN
    if (!b || trial_steps < 1) return fail(GOM_E_ARG, "gom_batch_autotune: bad arguments");
    for (int32_t i = 0; i < b->count; ++i)
        if (b->subs[(size_t)i]->open_next >= 0)
            return fail(GOM_E_STATE, "gom_batch_autotune: instance %d has an open generation",
                        i);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GOM_E_DEVICE, "gom_batch_autotune: %s", hipGetErrorString(he));
    }
    int rc = GOM_OK;
    hipError_t e = hipSuccess;
    // time `trial_steps` steps under each (narrow, class-launch) pair, two interleaved rounds
    auto tune = [&](const std::vector<std::pair<int64_t, int64_t>> &cands) {
        std::vector<double> total(cands.size(), 0.0);
        for (int round = 0; round < 2 && rc == GOM_OK && e == hipSuccess; ++round) {
            for (size_t q = 0; q < cands.size() && rc == GOM_OK && e == hipSuccess; ++q) {
                rc = batch_regroup(b, cands[q].first, cands[q].second, st);
                if (rc) break;
                e = hipEventRecord(e0, st);
                for (int32_t t = 0; t < trial_steps && e == hipSuccess && rc == GOM_OK; ++t) {
                    e = launch_batch_step(b->d_insts, b->count, b->d_blk, b->groups.data(),
                                          (int)b->groups.size(), b->d_vblk, b->vblocks,
                                          bcl_plan(b), st);
                    if (e == hipSuccess) rc = batch_solo_steps(b, 1, st);
                }
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                total[q] += ms;
                b->g_done += trial_steps;
            }
        }
        return cands[(size_t)(std::min_element(total.begin(), total.end()) - total.begin())];
    };
    // first which instances take the batched class launches (with the current block sizes),
    // then the resident block sizes of the others
    std::vector<std::pair<int64_t, int64_t>> c1;
    for (int64_t m : distinct_thresholds(b, {-1, 50000, 20000, 5000, 0}, true))
        c1.push_back({b->narrow_max_n, m});
    std::pair<int64_t, int64_t> best = tune(c1);
    if (rc == GOM_OK && e == hipSuccess) {
        std::vector<std::pair<int64_t, int64_t>> c2;
        for (int64_t nm : distinct_thresholds(b, {-1, 2048, 8192, 16384, 32768, (int64_t)1 << 40},
                                              false))
            c2.push_back({nm, best.second});
        best = tune(c2);
    }
    // then the class launches' positions per wave (when some instance takes them)
    rc = rc == GOM_OK && e == hipSuccess ? batch_regroup(b, best.first, best.second, st) : rc;
    if (rc == GOM_OK && e == hipSuccess && !b->bcl.empty()) {
        // (the bit-sliced form when admitted, else lane = solution with 1, 2, 4, 8 positions)
        const int gsv[] = {1, 0, 0, 0, 0}, ppws[] = {b->bcl_ppw, 1, 2, 4, 8};
        const int q0 = b->bcl_gs_ok ? 0 : 1;
        std::vector<double> total(5, 0.0);
        total[0] = b->bcl_gs_ok ? 0.0 : 1e300;
        for (int round = 0; round < 2 && rc == GOM_OK && e == hipSuccess; ++round)
            for (int q = q0; q < 5 && rc == GOM_OK && e == hipSuccess; ++q) {
                b->bcl_gs_use = gsv[q] != 0;
                b->bcl_ppw = ppws[q];
                // (the form decides whether univariate instances take the class launches)
                rc = batch_regroup(b, best.first, best.second, st);
                if (rc) break;
                e = hipEventRecord(e0, st);
                for (int32_t t = 0; t < trial_steps && e == hipSuccess && rc == GOM_OK; ++t) {
                    e = launch_batch_step(b->d_insts, b->count, b->d_blk, b->groups.data(),
                                          (int)b->groups.size(), b->d_vblk, b->vblocks,
                                          bcl_plan(b), st);
                    if (e == hipSuccess) rc = batch_solo_steps(b, 1, st);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                total[(size_t)q] += ms;
                b->g_done += trial_steps;
            }
        const size_t qb = (size_t)(std::min_element(total.begin(), total.end()) - total.begin());
        b->bcl_gs_use = gsv[qb] != 0;
        b->bcl_ppw = ppws[qb];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess)
        return fail(GOM_E_DEVICE, "gom_batch_autotune: %s", hipGetErrorString(e));
    rc = batch_regroup(b, best.first, best.second, st);
    if (rc) return rc;
    // the trial steps advanced the instances: keep the host's generation counts in step
    HIP_TRY(batch_snapshot(b, 0, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t i = 0; i < b->count; ++i) b->subs[(size_t)i]->g_host = b->h_st[i].generation;
    if (narrow_out) *narrow_out = best.first;
    if (class_min_out) *class_min_out = best.second;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_batch_set_class_launch(gom_batch *b, int64_t min_n, void *stream) {
    GUARD_BEGIN
    if (!b) return fail(GOM_E_ARG, "gom_batch_set_class_launch: null batch");
    return batch_regroup(b, b->narrow_max_n, min_n, (hipStream_t)stream);
    GUARD_END
}

extern "C" int gom_batch_get_class_launch(const gom_batch *b, int64_t *min_n, int32_t *instances,
                                          int32_t *launches, int32_t *positions_per_wave) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_get_class_launch: null batch");
    if (min_n) *min_n = b->bcl_min_n;
    if (instances) *instances = (int32_t)b->bcl.size();
    if (launches) *launches = b->bcl.empty() ? 0 : b->bcl_kmax;
    if (positions_per_wave) *positions_per_wave = b->bcl_ppw;
    return GOM_OK;
}

extern "C" int gom_batch_set_class_bitsliced(gom_batch *b, int enabled, void *stream) {
    GUARD_BEGIN
    if (!b) return fail(GOM_E_ARG, "gom_batch_set_class_bitsliced: null batch");
    b->bcl_gs_use = enabled != 0;
    // (which instances take the class launches depends on the form)
    return batch_regroup(b, b->narrow_max_n, b->bcl_min_n, (hipStream_t)stream);
    GUARD_END
}

extern "C" int gom_batch_get_class_bitsliced(const gom_batch *b, int *enabled, int *available) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_get_class_bitsliced: null batch");
    if (enabled) *enabled = b->bcl_gs_ok && b->bcl_gs_use;
    if (available) *available = b->bcl_gs_ok;
    return GOM_OK;
}

extern "C" int gom_batch_set_class_positions(gom_batch *b, int32_t positions_per_wave) {
    if (!b) return fail(GOM_E_ARG, "gom_batch_set_class_positions: null batch");
    if (positions_per_wave < 1 || positions_per_wave > kBclPositions)
        return fail(GOM_E_RANGE, "gom_batch_set_class_positions: %d (1..%d)", positions_per_wave,
                    kBclPositions);
    b->bcl_ppw = positions_per_wave;
    drop_graph(b);
    return GOM_OK;
}

extern "C" int gom_batch_state(gom_batch *b, int32_t index, gom_state **state) {
    if (!b || !state || index < 0 || index >= b->count)
        return fail(GOM_E_ARG, "gom_batch_state: bad arguments");
    *state = b->subs[(size_t)index];
    return GOM_OK;
}

// ------------------------------------------------------------------------------------------
// Serving loop: jobs arrive at any time, are admitted first come first served while their
// states fit in the server's arena, and advance independently: each admitted job runs on one
// of a few streams (the least loaded at admission), a chunk of generations at a time, and its
// next chunk is enqueued as soon as the previous chunk's run scalars have reached the host.
// Jobs on different streams overlap on the device.  A job's random numbers depend only on
// its seed, so its result does not depend on what else is running.
// ------------------------------------------------------------------------------------------
namespace {

struct ServerJob {
    int64_t id = 0;
    const mc_graph *g = nullptr;
    const gom_fos *f = nullptr;
    int32_t pop = 0, max_gens = 0;
    uint64_t seed = 0;
    int64_t target = 0;
    int rule = 0, order = 0;
    size_t bytes = 0, off = 0;
    gom_state *s = nullptr;
    int lane = 0;
    bool large = false;       // runs alone on lane 0 (size-aware placement)
    int slot = 0;             // chunk slot (event, snapshot) the next chunk uses
    int oldest = 0;           // slot of the oldest chunk in flight
    int pending = 0;          // chunks in flight (at most two: one runs while one waits)
    bool finishing = false;   // finished (target or limit); waits for its last chunk
    DevState last{};          // the run scalars when it finished
    bool retired = false;     // finished: result recorded, state and memory released
    double submit_ms = 0.0, admit_ms = 0.0;
};

}  // namespace

struct gom_server {
    char *arena = nullptr;
    size_t bytes = 0;
    int32_t max_jobs = 0, chunk = 4;
    std::vector<hipStream_t> lanes;       // owned streams (default priority)
    std::vector<int32_t> lane_jobs;
    int64_t large_min_n = -1;             // jobs with at least this many vertices are large
                                          // (-1: no distinction)
    int32_t large_active = 0;
    ArenaBlocks blocks;                   // first-fit, coalescing
    std::deque<ServerJob> queue;
    std::vector<ServerJob> active;
    std::vector<gom_job_result> done;
    int64_t next_id = 0;
    std::chrono::steady_clock::time_point t0;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

extern "C" void gom_server_free(gom_server *sv) {
    if (!sv) return;
    for (hipStream_t q : sv->lanes) (void)hipStreamSynchronize(q);
    for (ServerJob &J : sv->active)
        if (!J.retired) gom_state_free(J.s);
    for (hipStream_t q : sv->lanes) (void)hipStreamDestroy(q);
    delete sv;
}

extern "C" int gom_server_create(void *dev_arena, size_t arena_bytes, int32_t max_jobs,
                                 int32_t streams, gom_server **out) {
    GUARD_BEGIN
    if (!dev_arena || !out || max_jobs < 1 || streams < 1 || streams > 16)
        return fail(GOM_E_ARG, "gom_server_create: bad arguments");
    if ((reinterpret_cast<uintptr_t>(dev_arena) & 255) != 0)
        return fail(GOM_E_NOMEM, "gom_server_create: arena must be 256-byte aligned");
    if (arena_bytes < 256) return fail(GOM_E_NOMEM, "gom_server_create: arena too small");
    auto *sv = new gom_server;
    sv->arena = (char *)dev_arena;
    sv->bytes = arena_bytes & ~(size_t)255;
    sv->max_jobs = max_jobs;
    sv->blocks.reset(sv->bytes);
    sv->t0 = std::chrono::steady_clock::now();
    for (int32_t q = 0; q < streams; ++q) {
        hipStream_t h = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&h, hipStreamNonBlocking);
        if (e != hipSuccess) {
            gom_server_free(sv);
            return fail(GOM_E_DEVICE, "gom_server_create: %s", hipGetErrorString(e));
        }
        sv->lanes.push_back(h);
    }
    sv->lane_jobs.assign((size_t)streams, 0);
    *out = sv;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_server_set_large(gom_server *sv, int64_t large_min_n) {
    if (!sv) return fail(GOM_E_ARG, "gom_server_set_large: null server");
    sv->large_min_n = large_min_n;
    return GOM_OK;
}

extern "C" int gom_server_submit(gom_server *sv, const mc_graph *g, const gom_fos *f,
                                 int32_t pop, uint64_t seed, int64_t target,
                                 int32_t max_generations, int neutral_rule, int class_order,
                                 int64_t *job) {
    GUARD_BEGIN
    if (!sv || !g || !f || !job || max_generations < 0)
        return fail(GOM_E_ARG, "gom_server_submit: bad arguments");
    ServerJob J;
    int rc = gom_state_bytes(g, f, pop, &J.bytes);
    if (rc) return rc;
    if (align_up(J.bytes) > sv->bytes)
        return fail(GOM_E_NOMEM, "gom_server_submit: the job needs %zu bytes, more than the "
                    "whole arena", J.bytes);
    if (neutral_rule != GOM_NEUTRAL_PAPER && neutral_rule != GOM_NEUTRAL_ALWAYS)
        return fail(GOM_E_ARG, "gom_server_submit: unknown neutral rule %d", neutral_rule);
    if (class_order != GOM_ORDER_RANDOM && class_order != GOM_ORDER_FIXED)
        return fail(GOM_E_ARG, "gom_server_submit: unknown class order %d", class_order);
    J.id = sv->next_id++;
    J.g = g;
    J.f = f;
    J.pop = pop;
    J.seed = seed;
    J.target = target;
    J.max_gens = max_generations;
    J.rule = neutral_rule;
    J.order = class_order;
    J.submit_ms = sv->now_ms();
    sv->queue.push_back(J);
    *job = J.id;
    return GOM_OK;
    GUARD_END
}

namespace {

// Enqueue the job's next chunk of generations and the copy of its run scalars.
// The job's next chunk of generations and the snapshot of its run scalars, in the next slot;
// nothing once its generation limit has been enqueued (but a snapshot when no chunk is in
// flight, so that a job with no generation left still reports).  A generation enqueued after the target
// was reached does nothing on the device, so a job keeps two chunks in flight: the next one
// is queued while the last one runs, and no host round trip separates them.
int server_issue(gom_server *sv, ServerJob &J) {
    gom_state *s = J.s;
    hipStream_t q = sv->lanes[(size_t)J.lane];
    const int32_t n = std::min(sv->chunk, J.max_gens - s->g_host);
    if (n <= 0 && J.pending > 0) return GOM_OK;  // (with none in flight: a snapshot alone)
    for (int32_t t = 0; t < n; ++t) {
        int rc = enqueue_generation(s, s->g_host, J.target, q);
        if (rc) return rc;
        s->g_host++;
    }
    HIP_TRY(hipMemcpyAsync(&s->h_st[J.slot], s->d_st, sizeof(DevState), hipMemcpyDeviceToHost,
                           q));
    HIP_TRY(hipEventRecord(s->chunk_ev[J.slot], q));
    J.slot ^= 1;
    J.pending++;
    return GOM_OK;
}

}  // namespace

extern "C" int gom_server_step(gom_server *sv, int32_t *n_active, int32_t *n_queued) {
    GUARD_BEGIN
    if (!sv) return fail(GOM_E_ARG, "gom_server_step: null server");
    // admission, first come first served while the arena has room; with size-aware
    // placement a large job waits (without holding back the small jobs behind it) while
    // another large job runs, and runs alone on lane 0, the small jobs on the other lanes
    const bool sized = sv->large_min_n >= 0 && sv->lanes.size() >= 2;
    size_t qi = 0;
    while (qi < sv->queue.size() && (int32_t)sv->active.size() < sv->max_jobs) {
        ServerJob &J = sv->queue[qi];
        J.large = sized && (int64_t)J.g->n >= sv->large_min_n;
        if (J.large && sv->large_active > 0) {
            ++qi;
            continue;
        }
        size_t off = 0;
        if (!sv->blocks.alloc(J.bytes, &off)) break;
        int lane = 0;
        if (sized) {
            lane = J.large ? 0 : 1;
            for (int q = 2; q < (int)sv->lanes.size() && !J.large; ++q)
                if (sv->lane_jobs[(size_t)q] < sv->lane_jobs[(size_t)lane]) lane = q;
        } else {
            for (int q = 1; q < (int)sv->lanes.size(); ++q)
                if (sv->lane_jobs[(size_t)q] < sv->lane_jobs[(size_t)lane]) lane = q;
        }
        gom_state *s = nullptr;
        int rc = gom_state_init(J.g, J.f, J.pop, J.seed, J.rule, J.order, sv->arena + off,
                                align_up(J.bytes), sv->lanes[(size_t)lane], &s);
        if (rc) {
            // the job cannot start: it leaves the queue with a failed result, so that the
            // jobs behind it are still admitted
            sv->blocks.release(off, J.bytes);
            gom_job_result r{};
            r.job = J.id;
            r.status = rc;
            r.submit_ms = J.submit_ms;
            r.admit_ms = r.done_ms = sv->now_ms();
            sv->done.push_back(r);
            sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)qi);
            continue;
        }
        // jobs share the device: a fused sweep's chunks wait for each other, which needs all
        // of its blocks on the device at once, so served jobs sweep class by class
        s->fused_use = false;
        J.s = s;
        J.off = off;
        J.lane = lane;
        sv->lane_jobs[(size_t)lane]++;
        if (J.large) sv->large_active++;
        J.admit_ms = sv->now_ms();
        sv->active.push_back(J);
        sv->queue.erase(sv->queue.begin() + (std::ptrdiff_t)qi);
        rc = server_issue(sv, sv->active.back());
        if (rc == GOM_OK) rc = server_issue(sv, sv->active.back());
        if (rc) return rc;
    }
    // progress: every job whose chunk has finished is retired or given its next chunk; a
    // retired job is marked at once and leaves the active list however this pass ends
    RetiredSweep<ServerJob> sweep{sv->active};
    for (ServerJob &J : sv->active) {
        gom_state *s = J.s;
        // every finished chunk, oldest first: a job not yet finished gets its next chunk
        while (J.pending > 0) {
            const hipError_t qe = hipEventQuery(s->chunk_ev[J.oldest]);
            if (qe == hipErrorNotReady) break;
            HIP_TRY(qe);
            const DevState h = s->h_st[J.oldest];
            J.oldest ^= 1;
            J.pending--;
            if (J.finishing) continue;
            if (h.elite_fitness >= J.target || h.generation >= J.max_gens) {
                J.finishing = true;
                J.last = h;
            } else {
                int rc = server_issue(sv, J);
                if (rc) return rc;
            }
        }
        if (!J.finishing || J.pending > 0) continue;  // (its last chunk still runs)
        const DevState h = J.last;
        gom_job_result r{};
        r.job = J.id;
        r.status = GOM_OK;
        r.generations = h.generation;
        r.reached = h.elite_fitness >= J.target ? 1 : 0;
        r.best = h.elite_fitness;
        r.attempted = (int64_t)s->N * s->n_sets * (int64_t)h.generation;
        r.evaluated = h.evaluated;
        r.accepted = h.accepted;
        r.submit_ms = J.submit_ms;
        r.admit_ms = J.admit_ms;
        r.done_ms = sv->now_ms();
        int rc = gom_state_hash(s, sv->lanes[(size_t)J.lane], &r.hash);
        if (rc) return rc;
        sv->done.push_back(r);
        gom_state_free(s);
        J.s = nullptr;
        J.retired = true;
        sv->blocks.release(J.off, J.bytes);
        sv->lane_jobs[(size_t)J.lane]--;
        if (J.large) sv->large_active--;
    }
    if (n_active) *n_active = (int32_t)sv->active.size() - (int32_t)std::count_if(
        sv->active.begin(), sv->active.end(), [](const ServerJob &J) { return J.retired; });
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_server_results(gom_server *sv, gom_job_result *out, int32_t capacity,
                                  int32_t *n) {
    if (!sv || !n || (capacity > 0 && !out)) return fail(GOM_E_ARG, "gom_server_results: bad arguments");
    const int32_t k = std::min<int32_t>(capacity, (int32_t)sv->done.size());
    std::copy(sv->done.begin(), sv->done.begin() + k, out);
    sv->done.erase(sv->done.begin(), sv->done.begin() + k);
    *n = k;
    return GOM_OK;
}

extern "C" int gom_server_info(const gom_server *sv, int32_t *n_active, int32_t *n_queued,
                               int32_t *n_streams, size_t *free_bytes) {
    if (!sv) return fail(GOM_E_ARG, "gom_server_info: null server");
    if (n_active) *n_active = (int32_t)sv->active.size();
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    if (n_streams) *n_streams = (int32_t)sv->lanes.size();
    if (free_bytes) *free_bytes = sv->blocks.free_bytes();
    return GOM_OK;
}

// ------------------------------------------------------------------------------------------
// Interleaved Multi-start Scheme (Section 6.3): populations of n_base * 2^(i-1) solutions,
// level i seeded with seed + i - 1, each in its own part of the arena; a step runs one
// generation of level 1 and, whenever level i has then completed a multiple of c_ims
// generations, one generation of level i + 1 (created at its first generation).  The run
// ends after the step in which some level's elitist reached the target, or when the
// generation budget is spent.  The populations are independent, so each level's trajectory
// is that of its own solo run.
// ------------------------------------------------------------------------------------------
extern "C" int gom_ims_bytes(const mc_graph *g, const gom_fos *f, int32_t n_base,
                             int32_t max_levels, size_t *bytes) {
    GUARD_BEGIN
    if (!g || !f || !bytes || max_levels < 1 || max_levels > GOM_IMS_MAX_LEVELS || n_base < 2)
        return fail(GOM_E_ARG, "gom_ims_bytes: bad arguments");
    if (((int64_t)n_base << (max_levels - 1)) > GOM_MAX_POP)
        return fail(GOM_E_RANGE, "gom_ims_bytes: the largest level would hold %lld solutions "
                    "(at most %d)", (long long)((int64_t)n_base << (max_levels - 1)), GOM_MAX_POP);
    size_t o = 0;
    for (int32_t l = 0; l < max_levels; ++l) {
        size_t b = 0;
        int rc = gom_state_bytes(g, f, n_base << l, &b);
        if (rc) return rc;
        o = align_up(o + b);
    }
    *bytes = o;
    return GOM_OK;
    GUARD_END
}

extern "C" int gom_ims_run(const mc_graph *g, const gom_fos *f, int32_t n_base, int32_t c_ims,
                           int32_t max_levels, uint64_t seed, int neutral_rule,
                           int forced_improvement, int64_t target,
                           int32_t max_total_generations, void *dev_arena, size_t arena_bytes,
                           void *stream, gom_ims_result *out, gom_state **states) {
    GUARD_BEGIN
    size_t need = 0;
    int rc = gom_ims_bytes(g, f, n_base, max_levels, &need);
    if (rc) return rc;
    if (!out || !dev_arena || c_ims < 1 || max_total_generations < 0)
        return fail(GOM_E_ARG, "gom_ims_run: bad arguments");
    if (arena_bytes < need)
        return fail(GOM_E_NOMEM, "gom_ims_run: arena has %zu bytes, needs %zu", arena_bytes,
                    need);
    hipStream_t st = (hipStream_t)stream;
    char *arena = (char *)dev_arena;
    std::vector<gom_state *> lv;
    std::vector<size_t> off((size_t)max_levels, 0);
    for (int32_t l = 1; l < max_levels; ++l) {
        size_t b = 0;
        rc = gom_state_bytes(g, f, n_base << (l - 1), &b);
        if (rc) return rc;
        off[(size_t)l] = align_up(off[(size_t)l - 1] + b);
    }
    auto cleanup = [&](int code) {
        for (gom_state *s : lv) gom_state_free(s);
        return code;
    };
    std::vector<int64_t> elite;  // elitist fitness per level after its last generation
    int32_t total = 0, steps = 0;
    bool stop = false;
    // the recursive step of the scheme, written as a loop over levels
    auto step = [&]() -> int {
        for (int32_t i = 1; i <= max_levels; ++i) {
            if (total >= max_total_generations) return GOM_OK;
            if ((int32_t)lv.size() < i) {
                size_t b = 0;
                int r = gom_state_bytes(g, f, n_base << (i - 1), &b);
                gom_state *s = nullptr;
                if (r == GOM_OK)
                    r = gom_state_init(g, f, n_base << (i - 1), seed + (uint64_t)(i - 1),
                                       neutral_rule, GOM_ORDER_RANDOM, arena + off[(size_t)i - 1],
                                       b, stream, &s);
                if (r == GOM_OK && forced_improvement) r = gom_state_set_fi(s, 1);
                if (r) {
                    if (s) gom_state_free(s);
                    return r;
                }
                lv.push_back(s);
                DevState h;
                r = read_scalars(s, st, &h);
                if (r) return r;
                elite.push_back(h.elite_fitness);
                if (h.elite_fitness >= target) {
                    stop = true;
                    return GOM_OK;
                }
            }
            gom_state *s = lv[(size_t)i - 1];
            int r = enqueue_generation(s, s->g_host, INT64_MAX, st);
            if (r) return r;
            s->g_host++;
            ++total;
            DevState h;
            r = read_scalars(s, st, &h);
            if (r) return r;
            elite[(size_t)i - 1] = h.elite_fitness;
            if (h.generation % c_ims != 0) return GOM_OK;
        }
        return GOM_OK;
    };
    while (total < max_total_generations && !stop) {
        rc = step();
        if (rc) return cleanup(rc);
        ++steps;
        for (int64_t e : elite) stop |= e >= target;
    }
    gom_ims_result r{};
    r.levels = (int32_t)lv.size();
    r.steps = steps;
    r.total_generations = total;
    r.best = INT64_MIN;
    for (size_t l = 0; l < lv.size(); ++l) {
        DevState h;
        rc = read_scalars(lv[l], st, &h);
        if (rc) return cleanup(rc);
        r.generations[l] = h.generation;
        r.evaluated += h.evaluated;
        r.accepted += h.accepted;
        if (h.elite_fitness > r.best) {
            r.best = h.elite_fitness;
            r.best_level = (int32_t)l + 1;
        }
    }
    r.reached = lv.empty() ? 0 : (r.best >= target ? 1 : 0);
    *out = r;
    if (states) {
        for (int32_t l = 0; l < max_levels; ++l)
            states[l] = l < (int32_t)lv.size() ? lv[(size_t)l] : nullptr;
    } else {
        for (gom_state *s : lv) gom_state_free(s);
    }
    return GOM_OK;
    GUARD_END
}
