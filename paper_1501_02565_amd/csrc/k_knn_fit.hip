// k_knn_fit.hip -- K nearest matches per match on the match graph and the
// per-match interpolation model (Algorithm 1, steps 4-6; Sec. 3.2-3.4).
//
// One wavefront per match s:
//  1. Dijkstra from s on the match graph.  The visited set lives in LDS:
//     entries e (tentative distance, lightest incident edge, CSR range)
//     owned by lane e % 64, and an open-addressing node table whose slots
//     hold a node and its entry in one word.  Several frontier nodes are
//     settled per step: a frontier node v
//     with tentative d(v) is final once d(v) <= dmin + lightest_edge(v),
//     where dmin is the smallest tentative distance on the frontier (no
//     unsettled node can still lower it).  The edges of all nodes settled in
//     a step are relaxed together, one lane per edge, in windows of 64
//     edges: a prefix sum of the settled nodes' degrees places their edge
//     segments, a prefix maximum over marked segment starts tells every lane
//     whose edge it holds.  Every CSR record carries the neighbour's CSR
//     range and lightest edge, so one round of global loads per window is
//     all a step needs.  Float sums are monotone, so the distances equal
//     those of a sequential Dijkstra in the same precision, and a settled
//     distance is never lowered again.
//  2. The search stops once at least K settled nodes lie strictly below the
//     frontier minimum: the K smallest (distance, index) pairs are then all
//     settled.  They are selected by a bitonic sort of packed
//     (distance bits, index) keys, which also fixes the order of the sums
//     below (deterministic results).  s itself is first, at distance 0.
//  3. Weights k = exp(-a d) (Eq. 1).  NW: kernel-weighted mean displacement.
//     LA: weighted least squares of Eq. (2) with weights k^2 (each equation
//     scaled by k) or k, solved about the weighted centroid of the
//     neighbours (a 2x2 system per displacement component).  The fit is
//     done in FP32; when the neighbourhood is ill-conditioned (eigenvalue
//     ratio of the weighted position covariance below fp64_route, or fewer
//     than 3 neighbours) it is re-accumulated and solved in FP64, where a
//     near-collinear neighbourhood (ratio <= deg_tau) falls back to NW.
//  Output per match: b00 b01 b10 b11 c0 c1 with flow(p) = B (p - p_s) + c.
//
// Wave-wide sums, minima and scans use DPP row operations (registers only,
// fixed combination order).  The workgroup is a single wavefront, whose LDS
// instructions execute in issue order, so phases that hand data between
// lanes through LDS only need to keep the compiler from reordering them.
//
// A source whose visited set outgrows the small LDS table is put on an
// overflow list and redone by a second launch with a larger table; if that
// overflows too, the match's model is zero and the pair's counters record
// it (epic_get_stats then reports EPIC_ERR_CAPACITY for the pair).
#include <type_traits>

#include "epic_dev.h"
#include "fit.h"
#include "wave.h"

namespace epic {

namespace {

// Home slot of node v in a table of hcap slots (multiplicative hash, then
// the product range reduction, so hcap need not be a power of two).
__device__ __forceinline__ u32 node_slot(int v, u32 hcap) {
    return (u32)(((u64)((u32)v * 2654435761u) * hcap) >> 32);
}

// Compiler-only ordering of the wavefront's LDS accesses (see above).
__device__ __forceinline__ void lds_order() { __asm__ __volatile__("" ::: "memory"); }

// Node table slot: the node in the high bits over its entry (EB bits; the
// all-ones entry marks a node that got no entry), all ones when empty.
// 256-entry tables pack both into 32 bits (nodes below 2^23 - 1), larger
// ones into 64.
template <int VCAP>
struct NodeSlot {
    using T = typename std::conditional<(VCAP <= 256), u32, u64>::type;
    static constexpr int EB = VCAP <= 256 ? 9 : 32;
    static constexpr T EMPTY = ~(T)0;
    static constexpr u32 NO_ENTRY = VCAP <= 256 ? 0x1ffu : 0xffffffffu;
    static_assert(VCAP <= 256 ? VCAP < 0x1ff : true, "entry field");
    __device__ static T pack(int v, u32 e) { return ((T)(u32)v << EB) | (T)e; }
    __device__ static int node(T w) { return (int)(w >> EB); }
    __device__ static u32 entry(T w) { return (u32)(w & (T)NO_ENTRY); }
};

template <int VCAP, bool F64>
struct KnnLds {
    static constexpr int HCAP = VCAP + VCAP / 2;   // node table slots (load at most 2/3)
    static constexpr int TW = 64;                 // edges per relaxation window (one per lane)
    using DT = typename std::conditional<F64, u64, u32>::type;     // distance bits
    using RT = typename std::conditional<F64, double, float>::type;
    using ST = typename NodeSlot<VCAP>::T;
    // entry e: tentative distance (2e) and lightest incident edge (2e + 1);
    // FP32 packs the edge's high 16 float bits over the degree (low 16 bits),
    // the CSR record's own word.  After the search: the sort keys.
    alignas(16) DT dm[2 * VCAP];
    // entry e: CSR start (FP64: and degree); after the search, the entry's node
    u32 rd[F64 ? 2 * VCAP : VCAP];
    ST htab[HCAP];                // node table
    int snode[F64 ? VCAP : 1];    // FP64: node of each sort key
    u32 head[TW];                 // (window stamp << 12) | (1 + entry) of the edge segment
                                  // starting at a window position
};

template <bool F64>
__device__ __forceinline__ typename std::conditional<F64, double, float>::type from_bits(
    typename std::conditional<F64, u64, u32>::type b) {
    if constexpr (F64) return dbits(b); else return __uint_as_float(b);
}
template <bool F64>
__device__ __forceinline__ typename std::conditional<F64, u64, u32>::type to_bits(
    typename std::conditional<F64, double, float>::type v) {
    if constexpr (F64) return bitsd(v); else return __float_as_uint(v);
}

// Distance and lightest edge of entry e (one LDS read).
template <int VCAP, bool F64>
__device__ __forceinline__ void read_dm(const KnnLds<VCAP, F64>& S, int e,
                                        typename KnnLds<VCAP, F64>::RT& d,
                                        typename KnnLds<VCAP, F64>::RT& mi) {
    if constexpr (F64) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(&S.dm[2 * e]);
        d = dbits(v.x);
        mi = dbits(v.y);
    } else {
        const uint2 v = *reinterpret_cast<const uint2*>(&S.dm[2 * e]);
        d = __uint_as_float(v.x);
        mi = __uint_as_float(v.y);
    }
}

// Value of v in lane (this lane xor j); j is a power of two below 64 that
// the callers' unrolled loops make a constant.
__device__ __forceinline__ u64 xor_lane_u64(u64 v, int j) {
    switch (j) {
        case 1: return wave::xor_lane<1>(v);
        case 2: return wave::xor_lane<2>(v);
        case 4: return wave::xor_lane<4>(v);
        case 8: return wave::xor_lane<8>(v);
        case 16: return wave::xor_lane<16>(v);
        default: return wave::xor_lane<32>(v);
    }
}

// Lanes l of a wavefront with bit j of l clear, as a mask (j a power of two
// below 64): 0x5555..., 0x3333..., 0x0f0f..., ...
__device__ __forceinline__ constexpr u64 low_lanes(int j) { return ~0ull / ((1ull << j) + 1ull); }

// Ascending bitonic sort of 64 E keys held in registers, key lane + 64 r in
// v[r] (E = 1 or 2).  Exchanges across lanes go through DPP, swizzle and
// permute moves; the distance-64 exchange swaps the two registers of a lane.
// Which lanes keep the smaller key of a pair is a lane mask fixed by the step.
template <int E>
__device__ __forceinline__ void bitonic_regs(u64 (&v)[2], int lane) {
#pragma unroll
    for (int k = 2; k <= 64 * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j == 64) {                  // k = 128: ascending everywhere
                const u64 a = v[0], b = v[1];
                const bool lt = a < b;
                v[0] = lt ? a : b;
                v[1] = lt ? b : a;
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const u64 a = v[r], b = xor_lane_u64(a, j);
                    // the lower index of an ascending pair (or the upper of a
                    // descending one) keeps the smaller key
                    const u64 asc = k < 64 ? low_lanes(k) : (((64 * r) & k) == 0 ? ~0ull : 0ull);
                    const bool keep_min = __builtin_amdgcn_inverse_ballot_w64(~(low_lanes(j) ^ asc));
                    v[r] = ((a < b) == keep_min) ? a : b;
                }
            }
        }
    }
}

// Processes source `s` of pair P; returns false when the visited set did not
// fit the table (nothing written then).
template <int VCAP, int KMAX, bool F64>
__device__ __forceinline__ bool knn_fit_one(const PairDev& P, const RunDev& run, int s, KnnLds<VCAP, F64>& S) {
    using LdsT = KnnLds<VCAP, F64>;
    using RT = typename LdsT::RT;
    const RT RINF = (RT)INFINITY;
    constexpr int HCAP = LdsT::HCAP;
    constexpr int TW = LdsT::TW;
    constexpr int Q = TW / 64;          // edges per lane per window
    constexpr int R = VCAP / 64;        // entries per lane
    using NS = NodeSlot<VCAP>;
    using ST = typename NS::T;
    static_assert(VCAP < 4096 && TW <= 128, "head mark layout");
    constexpr int RK = KMAX / 64;
    const int lane = threadIdx.x;
    const int K = P.K;
    const int keff = __builtin_amdgcn_readfirstlane(P.counters[C_KEFF]);
    ST* const htab = S.htab;
    u64* const keys = reinterpret_cast<u64*>(S.dm);       // sort keys, after the search
    EPIC_GLOBAL float* prm = gmem(P.params) + 6LL * s;
    // the match's own row, fetched now so that its latency hides behind the search
    const float4 me = gload(reinterpret_cast<const float4*>(P.matches) + s);
    // read once: the LDS ordering points below would make the compiler
    // reload it from the descriptor at every window
    const uint4* const adj = P.adj;

    // ------------------------------------------------------------ Dijkstra
    for (int i = lane; i < HCAP; i += 64) htab[i] = NS::EMPTY;
    for (int i = lane; i < TW; i += 64) S.head[i] = 0u;
    for (int i = lane; i < 2 * VCAP; i += 64) S.dm[i] = to_bits<F64>(RINF);
    for (int i = lane; i < (F64 ? 2 * VCAP : VCAP); i += 64) S.rd[i] = 0u;
    __syncthreads();
    if (lane == 0) {
        const u32 a = gmem(P.row_ptr)[s], b = gmem(P.row_ptr)[s + 1];
        S.dm[0] = 0;
        if constexpr (F64) {
            S.dm[1] = gmem(P.minin64)[s];
            S.rd[0] = a;
            S.rd[1] = b - a;
        } else {
            // (a degree above 16 bits stops the pair before this kernel)
            S.dm[1] = (gmem(P.minin)[s] & 0xffff0000u) | (b - a);
            S.rd[0] = a;
        }
        htab[node_slot(s, HCAP)] = NS::pack(s, 0u);
    }
    __syncthreads();

    int nvis = 1;               // entries in use (the same in every lane)
    int stamp = 0;              // relaxation windows so far (head marks)
    int nsettled = 0;           // settled entries (the same in every lane)
    bool ovf = false;
    // per group r: the lanes whose entry lane + 64 r is settled, as a lane
    // mask (uniform: the per-lane tests are mask selects, updates scalar)
    u64 smask[R];
#pragma unroll
    for (int r = 0; r < R; ++r) smask[r] = 0ull;
    // per group r: the raw (distance, lightest edge) bits and CSR range of
    // entry lane + 64 r, kept across steps as loaded
    using DT2 = typename std::conditional<F64, ulonglong2, uint2>::type;
    DT2 dmr[R];
    u32 deg[R];
    RT d[R], mi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        dmr[r].x = dmr[r].y = to_bits<F64>(RINF);
        deg[r] = 0u;
    }
    RT dstop = RINF;
    for (;;) {
        // nvis and nsettled are the same in every lane; readfirstlane lets
        // the compiler keep them (and the branches on them) scalar
        const int nv = __builtin_amdgcn_readfirstlane(nvis);
        nsettled = __builtin_amdgcn_readfirstlane(nsettled);
        // only the groups of 64 entries that are in use are read and
        // scanned (a uniform bound); d[r] of the others stays infinite
        const int ru = (nv + 63) >> 6;
        // entries not in use read as (inf, inf, 0, 0): the table is filled
        // with them at the start, so the reads need no predicate; groups
        // beyond ru keep those values from before the loop
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r < ru) {
                const int e = lane + 64 * r;
                dmr[r] = *reinterpret_cast<const DT2*>(&S.dm[2 * e]);
                if constexpr (F64) deg[r] = S.rd[2 * e + 1];
            }
            d[r] = from_bits<F64>(dmr[r].x);
            if constexpr (F64) {
                mi[r] = from_bits<F64>(dmr[r].y);
            } else {
                mi[r] = __uint_as_float(dmr[r].y & 0xffff0000u);
                deg[r] = dmr[r].y & 0xffffu;
            }
        }
        // frontier minimum (entries not in use are infinite)
        RT fmin = RINF;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const RT dv = __builtin_amdgcn_inverse_ballot_w64(smask[r]) ? RINF : d[r];
            if constexpr (F64) fmin = fmin < dv ? fmin : dv;
            else fmin = __uint_as_float(min(__float_as_uint(fmin), __float_as_uint(dv)));   // d >= 0
        }
        RT dmin;
        if constexpr (F64) dmin = wave::min(fmin); else dmin = wave::min_nonneg(fmin);
        // settled entries strictly below the frontier minimum (only counted
        // once enough entries are settled at all)
        int below = 0;
        if (nsettled >= keff) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < ru) below += __popcll(wave::ballot(d[r] < dmin) & smask[r]);
        }
        if (below >= keff || !(dmin < RINF)) {
            dstop = dmin;       // nodes settled at this point lie at or above dmin
            break;
        }
        // settle the final frontier nodes; their edges are relaxed below
        u64 newly[R];
        int my_edges = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            newly[r] = 0ull;
            if (r >= ru) continue;
            const int nin = nv - 64 * r;                       // entries of group r in use, >= 1
            const u64 valid = nin >= 64 ? ~0ull : (1ull << nin) - 1ull;
            newly[r] = wave::ballot(d[r] <= dmin + mi[r]) & valid & ~smask[r];
            nsettled += __popcll(newly[r]);
            smask[r] |= newly[r];
            if (__builtin_amdgcn_inverse_ballot_w64(newly[r])) my_edges += (int)deg[r];
        }
        const int incl = wave::incl_scan(my_edges);
        const int T = __builtin_amdgcn_readlane(incl, 63);
        int off[R];
        {
            int o = incl - my_edges;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                off[r] = o;
                if (r < ru && __builtin_amdgcn_inverse_ballot_w64(newly[r])) o += (int)deg[r];
            }
        }
        int carry_start = 0, carry_e = 0;
        for (int wb = 0; wb < T; wb += TW) {
            // mark the segments that start in this window; marks carry the
            // window's stamp, so stale ones from earlier windows are ignored
            // and the array is never cleared (except when the stamp wraps)
            if (++stamp == (1 << 20)) {
                for (int i = lane; i < TW; i += 64) S.head[i] = 0u;
                lds_order();
                stamp = 1;
            }
            const u32 stamp_hi = (u32)stamp << 12;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < ru && __builtin_amdgcn_inverse_ballot_w64(newly[r]) && deg[r] > 0u && off[r] >= wb &&
                    off[r] < wb + TW)
                    S.head[off[r] - wb] = stamp_hi | (u32)(lane + 64 * r + 1);
            lds_order();
            const int nq = min(Q, (T - wb + 63) >> 6);   // chunks of 64 edges in this window
            bool act[Q];
            int qe[Q], qst[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                act[q] = false;
                qe[q] = 0;
                qst[q] = 0;
                if (q < nq) {
                    act[q] = wb + 64 * q + lane < T;
                    const u32 hv = S.head[64 * q + lane];
                    // (window position, entry) of the last segment start at
                    // or before this lane, plus one (0: none in this chunk)
                    const u32 sc = wave::incl_max((hv >> 12) == (u32)stamp
                                                      ? ((u32)(64 * q + lane) << 12) | (hv & 0xfffu) : 0u);
                    if (sc != 0u) {
                        qst[q] = wb + (int)(sc >> 12);
                        qe[q] = (int)(sc & 0xfffu) - 1;
                    } else {
                        qst[q] = carry_start;
                        qe[q] = carry_e;
                    }
                    carry_start = __builtin_amdgcn_readlane(qst[q], 63);
                    carry_e = __builtin_amdgcn_readlane(qe[q], 63);
                }
            }
            // each lane's edges: source entry's CSR start and settled distance
            RT du[Q];
            u32 ei[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                RT unused;
                read_dm<VCAP, F64>(S, qe[q], du[q], unused);
                const u32 st = S.rd[F64 ? 2 * qe[q] : qe[q]];
                ei[q] = act[q] ? st + (u32)(wb + 64 * q + lane - qst[q]) : 0u;
            }
            uint4 rec[Q];
            RT cand[Q], nbm[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                rec[q] = gload(adj + ei[q]);
                if constexpr (F64) {
                    cand[q] = du[q] + gmem(P.adjw64)[ei[q]];
                    nbm[q] = dbits(gmem(P.nbmin64)[ei[q]]);
                } else {
                    // the record carries the neighbour's lightest edge rounded
                    // down to 16 bits: a lower bound, which is all the settle
                    // test needs
                    cand[q] = du[q] + __uint_as_float(rec[q].y);
                    nbm[q] = __uint_as_float(rec[q].w & 0xffff0000u);
                }
            }
            // find or claim each neighbour's table slot with one
            // compare-and-swap per probe: it returns an empty slot (this
            // lane claimed it, for now without an entry), a slot of v
            // (already there) or of another node (next slot).
            // res: 0 while probing, else 1 + slot, bit 30 set when this lane
            // claimed it; RES_IDLE for lanes without an edge.
            constexpr u32 RES_WON = 1u << 30, RES_IDLE = ~0u;
            u32 res[Q], hh[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                res[q] = act[q] ? 0u : RES_IDLE;
                hh[q] = node_slot((int)rec[q].x, HCAP);
            }
            for (int probe = 0; probe < HCAP; ++probe) {
                bool any = false;
#pragma unroll
                for (int q = 0; q < Q; ++q) any = any || res[q] == 0u;
                if (wave::ballot(any) == 0ull) break;
                ST prev[Q];             // all chunks' compare-and-swaps in flight together
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    prev[q] = res[q] == 0u ? atomicCAS(&htab[hh[q]], NS::EMPTY, NS::pack((int)rec[q].x, NS::NO_ENTRY))
                                           : (ST)0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (res[q] == 0u) {
                        res[q] = prev[q] == NS::EMPTY ? (hh[q] + 1u) | RES_WON
                               : NS::node(prev[q]) == (int)rec[q].x ? hh[q] + 1u : 0u;
                        hh[q] = hh[q] + 1u == (u32)HCAP ? 0u : hh[q] + 1u;
                    }
                }
            }
            {
                bool lost = false;
#pragma unroll
                for (int q = 0; q < Q; ++q) lost = lost || res[q] == 0u;
                if (wave::ballot(lost) != 0ull) ovf = true;
            }
            // new nodes get entries (with their distance and CSR range)
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const bool won = res[q] != RES_IDLE && (res[q] & RES_WON) != 0u;
                const u64 m = wave::ballot(won);
                const int e = nvis + wave::lanes_below(m);
                nvis += __popcll(m);
                if (won) {
                    const u32 hs = (res[q] & (RES_WON - 1u)) - 1u;
                    if (e < VCAP) {
                        S.dm[2 * e] = to_bits<F64>(cand[q]);
                        if constexpr (F64) {
                            S.dm[2 * e + 1] = to_bits<F64>(nbm[q]);
                            S.rd[2 * e] = rec[q].z;
                            S.rd[2 * e + 1] = rec[q].w;
                        } else {
                            S.dm[2 * e + 1] = rec[q].w;        // lightest edge bits over the degree
                            S.rd[e] = rec[q].z;
                        }
                        htab[hs] = NS::pack((int)rec[q].x, (u32)e);
                    }
                }
            }
            if (nvis > VCAP) ovf = true;
            lds_order();
            // relax the nodes that were already in the table
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (res[q] != RES_IDLE && res[q] != 0u && (res[q] & RES_WON) == 0u) {
                    const u32 e = NS::entry(htab[res[q] - 1u]);
                    if (e != NS::NO_ENTRY) atomicMin(&S.dm[2 * e], to_bits<F64>(cand[q]));
                }
            }
            lds_order();
        }
        if (ovf) break;
    }
    if (ovf) return false;

    // ---------------------------------------- select the K nearest (sorted)
    // Candidates: settled entries strictly below dstop, sorted in LDS: FP32
    // as packed (distance bits, index) words, FP64 as (distance bits, index)
    // pairs held in two arrays.
    // each entry's node, from the node table (slot -> node, slot -> entry),
    // into the CSR array, which the search no longer needs
    int* const node_of = reinterpret_cast<int*>(S.rd);
    __syncthreads();
    for (int h = lane; h < HCAP; h += 64) {
        const ST w = htab[h];
        const u32 e = NS::entry(w);
        if (w != NS::EMPTY && e < (u32)VCAP) node_of[e] = NS::node(w);
    }
    __syncthreads();                 // the distances (the keys' space) are in registers from here
    int nc = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool c = __builtin_amdgcn_inverse_ballot_w64(smask[r]) && d[r] < dstop;
        const u64 m = wave::ballot(c);
        const int pos = nc + wave::lanes_below(m);
        nc += __popcll(m);
        if (c) {
            const int e = lane + 64 * r;
            if constexpr (F64) {
                keys[pos] = bitsd(d[r]);
                S.snode[pos] = node_of[e];
            } else {
                keys[pos] = ((u64)__float_as_uint(d[r]) << 32) | (u32)node_of[e];
            }
        }
    }
    int p2 = 64;
    while (p2 < nc) p2 <<= 1;
    int knode[RK];
    RT kdist[RK];
    bool sorted = false;
    if constexpr (!F64 && VCAP <= 256) {
        // up to 128 keys (the usual case): sorted in registers
        static_assert(RK <= 2, "register sort holds two keys per lane");
        if (p2 <= 128) {
            __syncthreads();
            u64 v[2];
            v[0] = lane < nc ? keys[lane] : ~0ull;
            v[1] = lane + 64 < nc ? keys[lane + 64] : ~0ull;
            if (p2 == 64) bitonic_regs<1>(v, lane); else bitonic_regs<2>(v, lane);
#pragma unroll
            for (int r = 0; r < RK; ++r) {
                knode[r] = (int)(u32)v[r];
                kdist[r] = __uint_as_float((u32)(v[r] >> 32));
            }
            sorted = true;
        }
    }
    if (!sorted) {
        for (int i = nc + lane; i < p2; i += 64) {
            keys[i] = ~0ull;
            if constexpr (F64) S.snode[i] = 0x7fffffff;
        }
        __syncthreads();
        // each lane takes compare-exchange pairs (i, i + j): pair t has i = t
        // with a zero bit inserted at the position of j
        for (int k = 2; k <= p2; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = lane; t < (p2 >> 1); t += 64) {
                    const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                    const int ixj = i | j;
                    {
                        const u64 a = keys[i], b = keys[ixj];
                        const bool up = (i & k) == 0;
                        if constexpr (F64) {
                            const int na = S.snode[i], nb = S.snode[ixj];
                            const bool gt = a > b || (a == b && na > nb);
                            const bool lt = a < b || (a == b && na < nb);
                            if (up ? gt : lt) {
                                keys[i] = b;
                                keys[ixj] = a;
                                S.snode[i] = nb;
                                S.snode[ixj] = na;
                            }
                        } else {
                            // keys are distinct except the padding, whose swap is harmless
                            if ((a > b) == up) {
                                keys[i] = b;
                                keys[ixj] = a;
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int r = 0; r < RK; ++r) {
            const int jj = lane + 64 * r;
            const u64 kb = jj < p2 ? keys[jj] : ~0ull;
            if constexpr (F64) {
                knode[r] = jj < p2 ? S.snode[jj] : 0x7fffffff;
                kdist[r] = dbits(kb);
            } else {
                knode[r] = (int)(u32)kb;
                kdist[r] = __uint_as_float((u32)(kb >> 32));
            }
        }
    }
    const int n = min(keff, nc);
    if (P.dbg_knn_idx) {
#pragma unroll
        for (int r = 0; r < RK; ++r) {
            const int jj = lane + 64 * r;
            if (jj < K) {
                const bool ok = jj < n;
                gmem(P.dbg_knn_idx)[(long long)s * K + jj] = ok ? knode[r] : -1;
                gmem(P.dbg_knn_d)[(long long)s * K + jj] = ok ? (float)kdist[r] : __int_as_float(0x7f800000);
            }
        }
    }

    // ----------------------------------------------------------------- fit
    const float xm = me.x, ym = me.y;
    const float um = me.z - xm, vm = me.w - ym;
    // the K nearest rows, all loads in flight at once (lanes beyond n load
    // the match's own row and do not use it)
    float4 mrow[RK];
#pragma unroll
    for (int r = 0; r < RK; ++r) {
        const int node = lane + 64 * r < n ? knode[r] : s;
        mrow[r] = gload(reinterpret_cast<const float4*>(P.matches) + node);
    }
    const bool la = P.mode == 1 && !run.force_nw;
    const FitOut fo = fit_about<RK, F64>(lane, n, kdist, mrow, xm, ym, um, vm, (double)me.z - (double)xm,
                                         (double)me.w - (double)ym, P.a, run.la_wpow, la, run.fp64_route,
                                         run.deg_tau);
    const float* out = fo.p;
    if (fo.fp64) {
        if (F64 && lane < 6) {
            double v = fo.p64[0];
#pragma unroll
            for (int i = 1; i < 6; ++i) v = lane == i ? fo.p64[i] : v;
            gmem(P.params64)[6LL * s + lane] = v;
        }
        if (lane == 0) {
            if (la) atomicAdd(&P.counters[C_FP64], 1);
            if (fo.degenerate) atomicAdd(&P.counters[C_DEGENERATE], 1);
        }
    }
    if (lane < 6) {
        float v = out[0];
#pragma unroll
        for (int i = 1; i < 6; ++i) v = lane == i ? out[i] : v;
        prm[lane] = v;
    }
    if (run.prune_px > 0.0f && lane == 0) {
        // consistency check (first, NW pass): the NW field at this match's
        // pixel is its own model's constant, out[4], out[5]
        const double du = ((double)me.z - (double)me.x) - (double)out[4];
        const double dv = ((double)me.w - (double)me.y) - (double)out[5];
        P.fill[s] = sqrt(du * du + dv * dv) <= (double)run.prune_px ? 1u : 0u;
    }
    return true;
}

// Writes the model and debug rows of a match that is not a graph node.
__device__ __forceinline__ void knn_fit_inactive(const PairDev& P, int s) {
    const int lane = threadIdx.x;
    if (lane < 6) P.params[6LL * s + lane] = 0.0f;
    if (lane == 0) P.fill[s] = 0u;        // never kept by the consistency check
    if (P.dbg_knn_idx)
        for (int j = lane; j < P.K; j += 64) {
            P.dbg_knn_idx[(long long)s * P.K + j] = -1;
            P.dbg_knn_d[(long long)s * P.K + j] = __int_as_float(0x7f800000);
        }
}

__device__ __forceinline__ bool knn_active(const PairDev& P, int s) {
    // a pair whose graph overflowed its hash has incomplete adjacency: skip
    // it (its status already reports EPIC_ERR_CAPACITY)
    const bool graph_ok = (P.counters[C_OVERFLOW] & 1) == 0;
    const int sp = P.seed_pix[s];
    return graph_ok && sp >= 0 && label_at(P, sp) == (u32)s && P.counters[C_KEFF] > 0;
}

}  // namespace

// First launch: one block (one wavefront) per match of every pair.
// At most 80 scalar registers: with the 82 the compiler otherwise takes,
// the hardware's allocation granule leaves room for 7 wavefronts per SIMD,
// not 8 (the dispatcher's SGPR-full stall counter says so, with LDS, VGPRs
// and wave slots all free), and the last 832 of 8000 matches start only as
// the first ones end; at 78 all of them start at once.
template <int VCAP, int KMAX, bool F64>
__global__ __launch_bounds__(64) __attribute__((amdgpu_num_sgpr(80))) void k_knn_fit(
    const PairDev* __restrict__ pairs, RunDev run) {
    __shared__ KnnLds<VCAP, F64> S;
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].src_block_base; });
    const PairDev& P = pairs[p];
    const int s = (int)blockIdx.x - P.src_block_base;
    if (s >= P.N) return;          // after the consistency check: a match that was removed
    if (!knn_active(P, s)) {
        knn_fit_inactive(P, s);
        return;
    }
    if (!knn_fit_one<VCAP, KMAX, F64>(P, run, s, S) && threadIdx.x == 0)
        run.ovf_list[atomicAdd(run.ovf_count, 1)] = (int)blockIdx.x;
}

// Second launch: the matches whose visited set did not fit, with a larger
// table.  A fixed grid walks the overflow list.
template <int VCAP, int KMAX, bool F64>
__global__ __launch_bounds__(64) void k_knn_fit_retry(const PairDev* __restrict__ pairs, RunDev run) {
    __shared__ KnnLds<VCAP, F64> S;
    const int count = *run.ovf_count;
    for (int i = (int)blockIdx.x; i < count; i += (int)gridDim.x) {
        const int gb = run.ovf_list[i];
        const int p = find_pair(run.npairs, gb, [&](int k) { return pairs[k].src_block_base; });
        const PairDev& P = pairs[p];
        const int s = gb - P.src_block_base;
        if (!knn_fit_one<VCAP, KMAX, F64>(P, run, s, S)) {
            knn_fit_inactive(P, s);
            if (threadIdx.x == 0) atomicOr(&P.counters[C_OVERFLOW], 2);
        }
        __syncthreads();
    }
}

namespace {
template <bool F64>
void launch_knn_t(const PairDev* d_pairs, const RunDev& run, int total_blocks, int kmax, int nmax, hipStream_t s) {
    const int retry_grid = 512;
    // 256-entry tables keep node and entry in one 32-bit slot (nodes below
    // 2^23 - 1); a call with larger pairs takes the 512-entry kernels
    const bool small_ids = nmax < (1 << 23) - 1;
    if (kmax <= 64 && small_ids) {
        hipLaunchKernelGGL((k_knn_fit<256, 64, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<1024, 64, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    } else if (kmax <= 128 && small_ids) {
        hipLaunchKernelGGL((k_knn_fit<256, 128, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<2048, 128, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    } else {
        hipLaunchKernelGGL((k_knn_fit<512, 256, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<2048, 256, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    }
}
}  // namespace

hipError_t launch_knn_fit(const PairDev* d_pairs, const RunDev& run, int total_blocks, int kmax, int nmax,
                          hipStream_t s) {
    if (run.precision == 1) launch_knn_t<true>(d_pairs, run, total_blocks, kmax, nmax, s);
    else launch_knn_t<false>(d_pairs, run, total_blocks, kmax, nmax, s);
    return hipGetLastError();
}

}  // namespace epic
