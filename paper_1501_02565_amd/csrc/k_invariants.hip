// k_invariants.hip -- device self-checks of a call's intermediate state, run
// when the context was created with debug_validate.  Each violated
// invariant adds to the pair's C_INVARIANT counter (one update per
// wavefront); the results themselves are not changed.
//
// Transform (one thread per pixel, after the transform):
//  * labels are defined: with usable matches, every pixel holds a finite
//    D >= 0 and the label of a match placed on a pixel;
//  * the fixpoint holds: no neighbour q offers p a better key than it holds,
//    in the transform's own arithmetic.  FP32: key(p) <= (D(q) + step(q, p),
//    L(q)) lexicographically.  FP64: D(p) <= D(q) + step(q, p), and L(p) is
//    the lowest label among p's tight predecessors (or p's own seed).  With
//    the seeds below this makes D the discrete geodesic distance of Eq. (3)
//    and L its lowest-index minimiser (Sec. 3.4);
//  * seeds: the pixel of a placed match has D = 0 and a label no higher
//    than the match's index, placed on that same pixel.
// Graph (one thread per CSR record, after the scatter):
//  * a record of m names a neighbour n != m with a finite weight >= 0, and
//    n's list holds m with the same weight bits (the adjacency is
//    symmetric);
//  * the record's copy of n's CSR start (and, on the FP32 path, degree)
//    agrees with the row pointers.
// debug_validate = 2 first raises pixel 0's distance of every pair by 1 (a
// planted violation the checks must report: a self-test of the checks; the
// call's results are then not meaningful).
#include "epic_dev.h"

namespace epic {

namespace {

__device__ __forceinline__ void count(const PairDev& P, bool bad) {
    const u64 b = __builtin_amdgcn_ballot_w64(bad);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&P.counters[C_INVARIANT], (int)__popcll(b));
}

// A match placed on pixel `pix` (the seeding's rule, read back).
__device__ __forceinline__ bool placed_on(const PairDev& P, u32 m, long long pix) {
    return m < (u32)P.N && (long long)P.seed_pix[m] == pix;
}

}  // namespace

__global__ __launch_bounds__(PIX_BLOCK) void k_plant(const PairDev* __restrict__ pairs, RunDev run) {
    const PairDev& P = pairs[blockIdx.x];
    if (threadIdx.x != 0 || P.H * P.W == 0) return;
    if (run.precision == 1) {
        P.keys[0] = bitsd(dbits(P.keys[0]) + 1.0);
    } else {
        const u64 k = P.keys[0];
        P.keys[0] = make_key(key_dist(k) + 1.0f, key_label(k));
    }
}

__global__ __launch_bounds__(PIX_BLOCK) void k_check_transform(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].pix_block_base; });
    const PairDev& P = pairs[p];
    const long long i = (long long)((int)blockIdx.x - P.pix_block_base) * PIX_BLOCK + threadIdx.x;
    const int H = P.H, W = P.W;
    const long long HW = (long long)H * W;
    const bool f64 = run.precision == 1;
    const bool usable = P.counters[C_USED] > 0;
    bool bad = false;
    if (i < HW && usable) {
        const int x = (int)(i % W), y = (int)(i / W);
        const u64 k = P.keys[i];
        const u32 lab = label_at(P, i);
        const double dp = f64 ? dbits(k) : (double)key_dist(k);
        // defined: finite D >= 0 and the label of a placed match
        if (!(dp >= 0.0 && dp < 1e300) || lab >= (u32)P.N || P.seed_pix[lab] < 0) {
            bad = true;
        } else {
            constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
            constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
            const float cp = P.cost[i];
            u32 best = placed_on(P, lab, i) ? lab : NO_LABEL;   // own seed, or a tight predecessor
            for (int d = 0; d < run.conn; ++d) {
                const int qx = x + DX[d], qy = y + DY[d];
                if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
                const long long q = (long long)qy * W + qx;
                const u64 kq = P.keys[q];
                if (f64) {
                    const double c = relax_f64(dbits(kq), step_f64(P.cost[q], cp, d));
                    if (c < dp) bad = true;
                    const u32 lq = P.labels[q];
                    if (c == dp && lq < best) best = lq;
                } else {
                    const float len = d < 4 ? 1.0f : 1.41421356237309515f;
                    const u64 cand = make_key(relax_f32(key_dist(kq), step_f32(len, P.cost[q], cp)), key_label(kq));
                    if (key_dist(kq) < INFINITY && cand < k) bad = true;
                }
            }
            if (f64 && best != lab) bad = true;
        }
    }
    // seeds, one match per thread of the pixel grid (strided when N > HW)
    const long long stride = (long long)((HW + PIX_BLOCK - 1) / PIX_BLOCK) * PIX_BLOCK;
    for (long long m = i; m < P.N; m += stride) {
        const int sp = P.seed_pix[m];
        if (sp < 0) continue;
        const u64 k = P.keys[sp];
        const u32 lab = label_at(P, sp);
        const bool zero = f64 ? k == 0ull : key_dist(k) == 0.0f;
        if (!zero || lab > (u32)m || !placed_on(P, lab, sp)) bad = true;
    }
    count(P, bad);
}

__global__ __launch_bounds__(SLOT_BLOCK) void k_check_graph(const PairDev* __restrict__ pairs, RunDev run) {
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].slot_block_base; });
    const PairDev& P = pairs[p];
    const long long r = (long long)((int)blockIdx.x - P.slot_block_base) * SLOT_BLOCK + threadIdx.x;
    const int N = P.N;
    const bool f64 = run.precision == 1;
    bool bad = false;
    // the graph exists once the scan accepted it (status 0)
    if (P.counters[C_STATUS] == 0 && N > 0 && r < (long long)P.row_ptr[N]) {
        // owner m of record r: the last row starting at or before r
        int lo = 0, hi = N - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((long long)P.row_ptr[mid] <= r) lo = mid; else hi = mid - 1;
        }
        const u32 m = (u32)lo;
        const uint4 rec = P.adj[r];
        const u32 n = rec.x;
        const float w = __uint_as_float(rec.y);
        if (n >= (u32)N || n == m || !(w >= 0.0f && w < INFINITY)) {
            bad = true;
        } else {
            const u32 rn = P.row_ptr[n], rn1 = P.row_ptr[n + 1];
            if (rec.z != rn || (!f64 && (rec.w & 0xffffu) != rn1 - rn) || (f64 && rec.w != rn1 - rn)) bad = true;
            bool found = false;
            for (u32 j = rn; j < rn1 && !found; ++j) {
                const uint4 back = P.adj[j];
                found = back.x == m && back.y == rec.y;
            }
            if (!found) bad = true;
        }
    }
    count(P, bad);
}

hipError_t launch_check_transform(const PairDev* d_pairs, const RunDev& run, int pix_blocks, int plant,
                                  hipStream_t s) {
    if (plant) hipLaunchKernelGGL(k_plant, dim3(run.npairs), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    hipLaunchKernelGGL(k_check_transform, dim3(pix_blocks), dim3(PIX_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

hipError_t launch_check_graph(const PairDev* d_pairs, const RunDev& run, int slot_blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_check_graph, dim3(slot_blocks), dim3(SLOT_BLOCK), 0, s, d_pairs, run);
    return hipGetLastError();
}

}  // namespace epic
