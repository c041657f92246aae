// k_knn_fit.hip -- K nearest matches per match on the match graph and the
// per-match interpolation model (Algorithm 1, steps 4-6; Sec. 3.2-3.4).
//
// One wavefront per match s:
//  1. Dijkstra from s on the match graph, with the visited set held in LDS
//     (open-addressing node -> entry table).  When a node enters the table
//     its adjacency range and lightest incident edge are fetched with it, so
//     each step needs one round of global loads (the settled nodes' packed
//     (neighbour, weight) edges).  Several frontier nodes are settled per
//     step: a frontier node v with tentative d(v) is final once
//     d(v) <= dmin + lightest_edge(v), where dmin is the smallest tentative
//     distance on the frontier (no unsettled node can still lower it).  The
//     edges of all nodes settled in a step are relaxed in parallel, one lane
//     per edge.  Float sums are monotone, so the distances equal those of a
//     sequential Dijkstra in the same precision.
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
// A source whose visited set outgrows the small LDS table is put on an
// overflow list and redone by a second launch with a table four times
// larger; only if that overflows too is the pair's status set.
#include <type_traits>

#include "epic_dev.h"

namespace epic {

namespace {

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}
__device__ __forceinline__ u32 node_slot(int v, int hbits) {
    return ((u32)v * 2654435761u) >> (32 - hbits);
}

template <int VCAP, bool F64>
struct KnnLds {
    static constexpr int HCAP = 2 * VCAP;
    using DT = typename std::conditional<F64, u64, u32>::type;     // distance bits
    using RT = typename std::conditional<F64, double, float>::type;
    int node[VCAP];
    DT dist[VCAP];
    DT minin[VCAP];          // lightest incident edge
    u32 rs[VCAP];            // adjacency start
    u32 deg[VCAP];
    unsigned char state[VCAP];   // 0 frontier, 1 settled
    unsigned short newly[VCAP];
    u64 buf[VCAP];           // node table (HCAP ints), then sort keys
    int snode[F64 ? VCAP : 1];   // FP64: node of each sort key
    unsigned short hidx[HCAP];
    int f_off[65];
    u32 f_start[64];
    RT f_d[64];
    int nvis, nnew, ncand, ovf;
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

// Loads a node's adjacency range and lightest edge into entry e.
template <int VCAP, bool F64>
__device__ __forceinline__ void fetch_node(const PairDev& P, int v, KnnLds<VCAP, F64>& S, int e) {
    const u32 a = P.row_ptr[v], b = P.row_ptr[v + 1];
    if constexpr (F64) S.minin[e] = P.minin64[v]; else S.minin[e] = P.minin[v];
    S.rs[e] = a;
    S.deg[e] = b - a;
}

// Processes source `s` of pair P; returns false when the visited set did not
// fit the table (nothing written then).
template <int VCAP, int KMAX, bool F64>
__device__ __forceinline__ bool knn_fit_one(const PairDev& P, const RunDev& run, int s, KnnLds<VCAP, F64>& S) {
    using RT = typename KnnLds<VCAP, F64>::RT;
    using DT = typename KnnLds<VCAP, F64>::DT;
    const RT RINF = (RT)INFINITY;
    constexpr int HCAP = KnnLds<VCAP, F64>::HCAP;
    constexpr int HBITS = (HCAP == 512) ? 9 : (HCAP == 1024) ? 10 : (HCAP == 2048) ? 11 : 12;
    static_assert((1 << HBITS) == HCAP, "hash size");
    constexpr int R = KMAX / 64;
    const int lane = threadIdx.x;
    const int K = P.K;
    const int keff = P.counters[C_KEFF];
    int* htab = reinterpret_cast<int*>(S.buf);
    float* prm = P.params + 6LL * s;

    // ------------------------------------------------------------ Dijkstra
    for (int i = lane; i < HCAP; i += 64) htab[i] = -1;
    __syncthreads();
    if (lane == 0) {
        S.nvis = 1;
        S.ovf = 0;
        S.node[0] = s;
        S.dist[0] = 0;
        S.state[0] = 0;
        fetch_node<VCAP, F64>(P, s, S, 0);
        const u32 h = node_slot(s, HBITS);
        htab[h] = s;
        S.hidx[h] = 0;
    }
    __syncthreads();

    RT dstop;
    for (;;) {
        const int nv = min(S.nvis, VCAP);
        RT dmin = RINF;
        for (int e = lane; e < nv; e += 64)
            if (S.state[e] == 0) dmin = fmin(dmin, from_bits<F64>(S.dist[e]));
        dmin = wave_min(dmin);
        if (lane == 0) S.nnew = 0;
        __syncthreads();
        // one scan: count settled nodes below dmin, settle the final ones
        int below = 0;
        for (int e = lane; e < nv; e += 64) {
            const RT d = from_bits<F64>(S.dist[e]);
            if (S.state[e] == 1) {
                below += d < dmin ? 1 : 0;
            } else if (d <= dmin + from_bits<F64>(S.minin[e])) {
                S.state[e] = 1;
                S.newly[atomicAdd(&S.nnew, 1)] = (unsigned short)e;
            }
        }
        below = wave_sum_i(below);
        __syncthreads();
        if (below >= keff || dmin == RINF || S.ovf) {
            dstop = dmin;    // nodes settled in this scan lie at or above dmin
            break;
        }
        const int nn = S.nnew;
        for (int base = 0; base < nn; base += 64) {
            const int cnt = min(64, nn - base);
            int dg = 0;
            if (lane < cnt) {
                const int e = S.newly[base + lane];
                dg = S.deg[e];
                S.f_start[lane] = S.rs[e];
                S.f_d[lane] = from_bits<F64>(S.dist[e]);
            }
            const int incl = wave_incl_scan(dg, lane);
            const int total = __shfl(incl, 63);
            if (lane < cnt) S.f_off[lane] = incl - dg;
            if (lane == 0) S.f_off[cnt] = total;
            __syncthreads();
            for (int j0 = 0; j0 < total; j0 += 64) {
                const int j = j0 + lane;
                const bool act = j < total;
                int v = -1;
                RT cand = 0;
                if (act) {
                    int lo = 0, hi = cnt - 1;       // last i with f_off[i] <= j
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (S.f_off[mid] <= j) lo = mid; else hi = mid - 1;
                    }
                    const u32 ei = S.f_start[lo] + (u32)(j - S.f_off[lo]);
                    const uint2 ed = P.adj[ei];
                    v = (int)ed.x;
                    if constexpr (F64) cand = S.f_d[lo] + P.adjw64[ei];
                    else cand = S.f_d[lo] + __uint_as_float(ed.y);
                }
                // phase A: find or claim v's slot
                int h = -1;
                bool won = false;
                if (act) {
                    u32 hh = node_slot(v, HBITS);
                    for (int probe = 0; probe < HCAP; ++probe) {
                        const int cur = htab[hh];
                        if (cur == v) { h = (int)hh; break; }
                        if (cur == -1) {
                            const int prev = atomicCAS(&htab[hh], -1, v);
                            if (prev == -1) { h = (int)hh; won = true; break; }
                            if (prev == v) { h = (int)hh; break; }
                        }
                        hh = (hh + 1u) & (u32)(HCAP - 1);
                    }
                    if (h < 0) S.ovf = 1;
                }
                // phase B: new nodes get an entry (with their adjacency range)
                if (won) {
                    const int e = atomicAdd(&S.nvis, 1);
                    if (e < VCAP) {
                        S.node[e] = v;
                        S.dist[e] = to_bits<F64>(RINF);
                        S.state[e] = 0;
                        fetch_node<VCAP, F64>(P, v, S, e);
                        S.hidx[h] = (unsigned short)e;
                    } else {
                        S.hidx[h] = 0xffff;
                        S.ovf = 1;
                    }
                }
                __syncthreads();
                // phase C: relax
                if (act && h >= 0) {
                    const int e = S.hidx[h];
                    if (e != 0xffff && S.state[e] == 0) atomicMin(&S.dist[e], to_bits<F64>(cand));
                }
                __syncthreads();
            }
        }
    }
    if (S.ovf) return false;

    // ---------------------------------------- select the K nearest (sorted)
    const int nv = min(S.nvis, VCAP);
    if (lane == 0) S.ncand = 0;
    __syncthreads();
    // sort keys: FP32 packs (distance bits, index) into one word; FP64 sorts
    // (distance bits, index) pairs held in two arrays
    auto key_node = [&](int j) -> int { if constexpr (F64) return S.snode[j]; else return (int)(u32)S.buf[j]; };
    auto key_dist = [&](int j) -> RT {
        if constexpr (F64) return dbits(S.buf[j]); else return __uint_as_float((u32)(S.buf[j] >> 32));
    };
    for (int e = lane; e < nv; e += 64) {
        const RT d = from_bits<F64>(S.dist[e]);
        if (S.state[e] == 1 && d < dstop) {
            const int pos = atomicAdd(&S.ncand, 1);
            if constexpr (F64) {
                S.buf[pos] = S.dist[e];
                S.snode[pos] = S.node[e];
            } else {
                S.buf[pos] = ((u64)S.dist[e] << 32) | (u32)S.node[e];
            }
        }
    }
    __syncthreads();
    const int nc = S.ncand;
    int p2 = 1;
    while (p2 < nc) p2 <<= 1;
    for (int i = nc + lane; i < p2; i += 64) {
        S.buf[i] = ~0ull;
        if constexpr (F64) S.snode[i] = 0x7fffffff;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < p2; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const u64 a = S.buf[i], b = S.buf[ixj];
                    const bool up = (i & k) == 0;
                    bool gt, lt;
                    if constexpr (F64) {
                        const int na = S.snode[i], nb = S.snode[ixj];
                        gt = a > b || (a == b && na > nb);
                        lt = a < b || (a == b && na < nb);
                    } else {
                        gt = a > b;
                        lt = a < b;
                    }
                    if (up ? gt : lt) {
                        S.buf[i] = b;
                        S.buf[ixj] = a;
                        if constexpr (F64) {
                            const int t = S.snode[i];
                            S.snode[i] = S.snode[ixj];
                            S.snode[ixj] = t;
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    const int n = min(keff, nc);
    if (P.dbg_knn_idx) {
        for (int j = lane; j < K; j += 64) {
            const bool ok = j < n;
            P.dbg_knn_idx[(long long)s * K + j] = ok ? key_node(j) : -1;
            P.dbg_knn_d[(long long)s * K + j] = ok ? (float)key_dist(j) : __int_as_float(0x7f800000);
        }
    }

    // ----------------------------------------------------------------- fit
    const float* M = P.matches;
    const float xm = M[4LL * s + 0], ym = M[4LL * s + 1];
    const float um = M[4LL * s + 2] - xm, vm = M[4LL * s + 3] - ym;
    const float a = P.a;
    const int wpow = run.la_wpow;
    float dx[R], dy[R], du[R], dv[R], kk[R], ww[R];
    float tk = 0.f, tu = 0.f, tv = 0.f, sw = 0.f, sx = 0.f, sy = 0.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = lane + 64 * r;
        dx[r] = dy[r] = du[r] = dv[r] = kk[r] = ww[r] = 0.f;
        if (j < n) {
            const int node = key_node(j);
            const float d = (float)key_dist(j);
            const float4 mn = *reinterpret_cast<const float4*>(M + 4LL * node);
            dx[r] = mn.x - xm;
            dy[r] = mn.y - ym;
            du[r] = (mn.z - mn.x) - um;
            dv[r] = (mn.w - mn.y) - vm;
            kk[r] = expf(-a * d);
            ww[r] = wpow == 1 ? kk[r] : kk[r] * kk[r];
            tk += kk[r];
            tu += kk[r] * du[r];
            tv += kk[r] * dv[r];
            sw += ww[r];
            sx += ww[r] * dx[r];
            sy += ww[r] * dy[r];
        }
    }
    tk = wave_sum(tk);
    tu = wave_sum(tu);
    tv = wave_sum(tv);
    float out[6] = {0.f, 0.f, 0.f, 0.f, um + tu / tk, vm + tv / tk};
    bool need64 = false;
    if (P.mode == 1) {
        sw = wave_sum(sw);
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        const float mx = sx / sw, my = sy / sw;
        float sxx = 0.f, sxy = 0.f, syy = 0.f, sxu = 0.f, syu = 0.f, sxv = 0.f, syv = 0.f, su = 0.f, sv = 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float ex = dx[r] - mx, ey = dy[r] - my, w = ww[r];
            sxx += w * ex * ex;
            sxy += w * ex * ey;
            syy += w * ey * ey;
            sxu += w * ex * du[r];
            syu += w * ey * du[r];
            sxv += w * ex * dv[r];
            syv += w * ey * dv[r];
            su += w * du[r];
            sv += w * dv[r];
        }
        sxx = wave_sum(sxx); sxy = wave_sum(sxy); syy = wave_sum(syy);
        sxu = wave_sum(sxu); syu = wave_sum(syu); sxv = wave_sum(sxv); syv = wave_sum(syv);
        su = wave_sum(su); sv = wave_sum(sv);
        const float det = sxx * syy - sxy * sxy;
        const float tr = sxx + syy;
        const float disc = sqrtf((sxx - syy) * (sxx - syy) + 4.0f * sxy * sxy);
        const float l1 = 0.5f * (tr + disc);
        const float ratio = l1 > 0.f ? (det / l1) / l1 : 0.f;
        need64 = F64 || n < 3 || !(ratio >= run.fp64_route);
        if (!need64) {
            const float b00 = (syy * sxu - sxy * syu) / det, b01 = (sxx * syu - sxy * sxu) / det;
            const float b10 = (syy * sxv - sxy * syv) / det, b11 = (sxx * syv - sxy * sxv) / det;
            out[0] = b00; out[1] = b01; out[2] = b10; out[3] = b11;
            out[4] = um + su / sw - (b00 * mx + b01 * my);
            out[5] = vm + sv / sw - (b10 * mx + b11 * my);
        }
    }
    if (F64) need64 = true;
    if (need64) {
        // FP64: re-accumulate from the inputs and solve (or fall back to NW)
        const double xmd = xm, ymd = ym;
        const double umd = (double)M[4LL * s + 2] - xmd, vmd = (double)M[4LL * s + 3] - ymd;
        double Dx[R], Dy[R], Du[R], Dv[R], Dw[R];
        double Tk = 0, Tu = 0, Tv = 0, Sw = 0, Sx = 0, Sy = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = lane + 64 * r;
            Dx[r] = Dy[r] = Du[r] = Dv[r] = Dw[r] = 0.0;
            if (j < n) {
                const int node = key_node(j);
                const double d = (double)key_dist(j);
                const double x = M[4LL * node + 0], y = M[4LL * node + 1];
                Dx[r] = x - xmd;
                Dy[r] = y - ymd;
                Du[r] = ((double)M[4LL * node + 2] - x) - umd;
                Dv[r] = ((double)M[4LL * node + 3] - y) - vmd;
                const double k = exp(-(double)a * d);
                Dw[r] = wpow == 1 ? k : k * k;
                Tk += k; Tu += k * Du[r]; Tv += k * Dv[r];
                Sw += Dw[r]; Sx += Dw[r] * Dx[r]; Sy += Dw[r] * Dy[r];
            }
        }
        Tk = wave_sum_d(Tk); Tu = wave_sum_d(Tu); Tv = wave_sum_d(Tv);
        double o[6] = {0, 0, 0, 0, umd + Tu / Tk, vmd + Tv / Tk};
        bool degenerate = false;
        if (P.mode == 1) {
            Sw = wave_sum_d(Sw); Sx = wave_sum_d(Sx); Sy = wave_sum_d(Sy);
            const double mx = Sx / Sw, my = Sy / Sw;
            double sxx = 0, sxy = 0, syy = 0, sxu = 0, syu = 0, sxv = 0, syv = 0, su = 0, sv = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double ex = Dx[r] - mx, ey = Dy[r] - my, w = Dw[r];
                sxx += w * ex * ex; sxy += w * ex * ey; syy += w * ey * ey;
                sxu += w * ex * Du[r]; syu += w * ey * Du[r];
                sxv += w * ex * Dv[r]; syv += w * ey * Dv[r];
                su += w * Du[r]; sv += w * Dv[r];
            }
            sxx = wave_sum_d(sxx); sxy = wave_sum_d(sxy); syy = wave_sum_d(syy);
            sxu = wave_sum_d(sxu); syu = wave_sum_d(syu); sxv = wave_sum_d(sxv); syv = wave_sum_d(syv);
            su = wave_sum_d(su); sv = wave_sum_d(sv);
            // covariance normalised by the weight sum; eigenvalues l1 >= l2
            const double cxx = sxx / Sw, cxy = sxy / Sw, cyy = syy / Sw;
            const double tr = cxx + cyy;
            const double disc = sqrt((cxx - cyy) * (cxx - cyy) + 4.0 * cxy * cxy);
            const double l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
            degenerate = n < 3 || !(l1 > 0.0) || l2 <= run.deg_tau * l1;
            if (!degenerate) {
                const double det = sxx * syy - sxy * sxy;
                const double b00 = (syy * sxu - sxy * syu) / det, b01 = (sxx * syu - sxy * sxu) / det;
                const double b10 = (syy * sxv - sxy * syv) / det, b11 = (sxx * syv - sxy * sxv) / det;
                o[0] = b00; o[1] = b01; o[2] = b10; o[3] = b11;
                o[4] = umd + su / Sw - (b00 * mx + b01 * my);
                o[5] = vmd + sv / Sw - (b10 * mx + b11 * my);
            }
        }
        for (int i = 0; i < 6; ++i) out[i] = (float)o[i];
        if (F64 && lane < 6) {
            double v = o[0];
#pragma unroll
            for (int i = 1; i < 6; ++i) v = lane == i ? o[i] : v;
            P.params64[6LL * s + lane] = v;
        }
        if (lane == 0) {
            if (P.mode == 1) atomicAdd(&P.counters[C_FP64], 1);
            if (degenerate) atomicAdd(&P.counters[C_DEGENERATE], 1);
        }
    }
    if (lane < 6) {
        float v = out[0];
#pragma unroll
        for (int i = 1; i < 6; ++i) v = lane == i ? out[i] : v;
        prm[lane] = v;
    }
    return true;
}

// Writes the model and debug rows of a match that is not a graph node.
__device__ __forceinline__ void knn_fit_inactive(const PairDev& P, int s) {
    const int lane = threadIdx.x;
    if (lane < 6) P.params[6LL * s + lane] = 0.0f;
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
template <int VCAP, int KMAX, bool F64>
__global__ __launch_bounds__(64) void k_knn_fit(const PairDev* __restrict__ pairs, RunDev run) {
    __shared__ KnnLds<VCAP, F64> S;
    const int p = find_pair(run.npairs, (int)blockIdx.x, [&](int i) { return pairs[i].src_block_base; });
    const PairDev& P = pairs[p];
    const int s = (int)blockIdx.x - P.src_block_base;
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
void launch_knn_t(const PairDev* d_pairs, const RunDev& run, int total_blocks, int kmax, hipStream_t s) {
    const int retry_grid = 512;
    if (kmax <= 64) {
        hipLaunchKernelGGL((k_knn_fit<256, 64, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<1024, 64, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    } else if (kmax <= 128) {
        hipLaunchKernelGGL((k_knn_fit<256, 128, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<2048, 128, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    } else {
        hipLaunchKernelGGL((k_knn_fit<512, 256, F64>), dim3(total_blocks), dim3(64), 0, s, d_pairs, run);
        hipLaunchKernelGGL((k_knn_fit_retry<2048, 256, F64>), dim3(retry_grid), dim3(64), 0, s, d_pairs, run);
    }
}
}  // namespace

hipError_t launch_knn_fit(const PairDev* d_pairs, const RunDev& run, int total_blocks, int kmax,
                          hipStream_t s) {
    if (run.precision == 1) launch_knn_t<true>(d_pairs, run, total_blocks, kmax, s);
    else launch_knn_t<false>(d_pairs, run, total_blocks, kmax, s);
    return hipGetLastError();
}

}  // namespace epic
