// k_prune.hip -- the consistency check of the matches (Sec. 5.1 of the
// paper, "Pruning of matches"): the interpolation is run once with the
// Nadaraya-Watson estimator, and the matches whose displacement differs from
// that first estimate at their own pixel by more than a threshold are
// removed before the interpolation proper.
//
// At the pixel of match m the NW field is the model of cell m, whose value
// there is its constant c_m, so the test only needs the per-match models of
// the first pass: m is kept when it was placed on its pixel and
// |u_m - c_m| <= threshold (Euclidean norm, evaluated in double from the
// FP32 model).  The K-NN + fit kernel of the first pass takes that decision
// right after the fit and leaves a flag per match; k_prune compacts the
// kept matches in index order (so ties keep breaking towards the lower
// original index) and points the pair's descriptor at them: the second
// pass of every kernel then sees N' matches.  The first pass's drop counts
// and status are saved in counters the second pass keeps.
#include "epic_dev.h"
#include "wave.h"

namespace epic {

// One workgroup of 1024 threads per pair: each thread owns a contiguous
// chunk of matches, counts its kept ones, and the counts are scanned
// (wavefront DPP scans, then across the 16 wavefronts) to place each kept
// match.
__global__ __launch_bounds__(1024) void k_prune(PairDev* __restrict__ pairs, RunDev run) {
    PairDev& P = pairs[blockIdx.x];
    __shared__ int s_wave[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = P.N;
    const int chunk = (N + 1023) / 1024;
    const int b = min(N, tid * chunk), e = min(N, b + chunk);
    const float4* rows = reinterpret_cast<const float4*>(P.matches);
    // keep flags left by the first pass's K-NN + fit (0 for matches that
    // were not placed on their pixel)
    auto keep = [&](int m) -> bool { return P.fill[m] != 0u; };
    int cnt = 0;
    for (int m = b; m < e; ++m) cnt += keep(m) ? 1 : 0;
    const int incl = wave::incl_scan(cnt);
    if (lane == 63) s_wave[wid] = incl;
    __syncthreads();
    int pos = incl - cnt;
    for (int w = 0; w < wid; ++w) pos += s_wave[w];
    for (int m = b; m < e; ++m) {
        if (!keep(m)) continue;
        gstore(reinterpret_cast<float4*>(P.matches_kept) + pos, gload(rows + m));
        P.kept_idx[pos] = m;
        if (P.dbg_kept) P.dbg_kept[pos] = m;
        ++pos;
    }
    int total = 0;
    for (int w = 0; w < 16; ++w) total += s_wave[w];
    __syncthreads();                 // every thread is done with the first pass's N and rows
    if (tid == 0) {
        int* c = P.counters;
        c[C_PRUNED] = c[C_USED] - total;
        c[C_OUTSIDE0] = c[C_OUTSIDE];
        c[C_DUP0] = c[C_DUPLICATE];
        // a first-pass model that a K-NN overflow left at zero decided a
        // match: report the capacity error of that pass
        c[C_STATUS0] = c[C_STATUS] != 0 ? c[C_STATUS] : ((c[C_OVERFLOW] & 2) ? -6 : 0);
        if (P.dbg_n_kept) *P.dbg_n_kept = total;
        P.N = total;
        P.matches = P.matches_kept;
    }
}

hipError_t launch_prune(PairDev* d_pairs, const RunDev& run, hipStream_t s) {
    hipLaunchKernelGGL(k_prune, dim3(run.npairs), dim3(1024), 0, s, d_pairs, run);
    return hipGetLastError();
}

}  // namespace epic
