/*
 * epic_ref.c -- plain FP64 CPU oracle for EpicFlow's sparse-to-dense,
 * edge-preserving interpolation (Revaud et al., "EpicFlow", Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant with the GPU library.
 *
 * It is deliberately slow and literal: binary-heap Dijkstra over pixels,
 * a sort-based boundary scan, binary-heap Dijkstra per match, Householder QR
 * for the affine fits, and a per-pixel assignment.  All arithmetic is double;
 * the cost map and matches are read as float and widened.
 *
 * Steps (the paper's Algorithm 1, Sec. 3.4):
 *   seeds     matches are pixels (Sec. 3.1); a match is placed on the pixel
 *             that contains it, matches outside the image are dropped and a
 *             pixel claimed by several matches keeps the lowest index.
 *   voronoi   geodesic distance, Eq. (3), discretised on the 8-connected
 *             (or 4-connected) pixel graph with step cost len*(C(p)+C(q))/2;
 *             D(p) = min over matches, L(p) = argmin with the lowest index
 *             winning ties (geodesic Voronoi cells, Sec. 3.4).
 *   graph     matches adjacent in L are joined; the weight is the geodesic
 *             distance restricted to the two cells (Sec. 3.4), computed as
 *             the minimum over adjacent pixel pairs (p in m, q in n) of
 *             D(p) + len*(C(p)+C(q))/2 + D(q).
 *   knn       N_K(p_m): the K matches nearest to p_m under Dijkstra on the
 *             graph, ordered by (distance, index); p_m itself is first.
 *   fit       weights k = exp(-a d) (Eq. 1).  NW: kernel-weighted mean
 *             displacement (Eq. 1).  LA: least squares of Eq. (2), each
 *             equation scaled by k (power 2 in the normal equations) or by
 *             sqrt(k) (power 1).  A near-collinear neighbourhood falls back
 *             to NW.
 *   assign    every pixel takes the model of its cell (Algorithm 1, final
 *             loop; Sec. 3.4 "Piecewise field"), output as displacement.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_INF (1.0 / 0.0)

/* ------------------------------------------------------------------ */
/* a binary min-heap of (key, tie, id) triples                          */
/* ------------------------------------------------------------------ */
typedef struct { double key; int tie; int id; } hitem;
typedef struct { hitem* a; long n, cap; } heap;

static int hless(const hitem* x, const hitem* y)
{
    return x->key < y->key || (x->key == y->key && x->tie < y->tie);
}

static void hpush(heap* h, double key, int tie, int id)
{
    if (h->n == h->cap) {
        h->cap = h->cap ? 2 * h->cap : 1024;
        h->a = (hitem*)realloc(h->a, (size_t)h->cap * sizeof(hitem));
    }
    long i = h->n++;
    hitem it = { key, tie, id };
    while (i > 0) {
        long p = (i - 1) / 2;
        if (!hless(&it, &h->a[p])) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = it;
}

static hitem hpop(heap* h)
{
    hitem top = h->a[0];
    hitem last = h->a[--h->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, s = i;
        const hitem* best = &last;
        if (l < h->n && hless(&h->a[l], best)) { s = l; best = &h->a[l]; }
        if (r < h->n && hless(&h->a[r], best)) { s = r; }
        if (s == i) break;
        h->a[i] = h->a[s];
        i = s;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* ------------------------------------------------------------------ */
/* pixel neighbourhoods                                                 */
/* ------------------------------------------------------------------ */
static const int NB_DX[8] = { 1, -1, 0, 0, 1, -1, 1, -1 };
static const int NB_DY[8] = { 0, 0, 1, -1, 1, 1, -1, -1 };
/* half-neighbourhood: every unordered adjacent pair is seen once, from the
 * pixel with the lower raster index */
static const int HALF_DX[4] = { 1, 0, 1, -1 };
static const int HALF_DY[4] = { 0, 1, 1, 1 };

static double step_len(int dx, int dy)
{
    return (dx != 0 && dy != 0) ? sqrt(2.0) : 1.0;
}

/* cost of the step between adjacent pixels p and q: the trapezoid rule for
 * the line integral of C along the segment (Eq. 3) */
static double step_cost(const float* C, long p, long q, int dx, int dy)
{
    return step_len(dx, dy) * (0.5 * ((double)C[p] + (double)C[q]));
}

void epic_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int epic_ref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* seeds: match -> pixel (or -1 when dropped)                           */
/* ------------------------------------------------------------------ */
int epic_ref_seeds(int H, int W, const float* matches, int N, int* seed_pix,
                   int* n_outside, int* n_duplicate)
{
    int* owner = (int*)malloc(sizeof(int) * (size_t)H * W);
    for (long i = 0; i < (long)H * W; ++i) owner[i] = -1;
    int used = 0, outside = 0, dup = 0;
    for (int m = 0; m < N; ++m) {
        double x = matches[4 * m + 0], y = matches[4 * m + 1];
        seed_pix[m] = -1;
        if (!isfinite(x) || !isfinite(y)) { ++outside; continue; }
        double fx = floor(x + 0.5), fy = floor(y + 0.5);
        if (fx < 0 || fy < 0 || fx >= W || fy >= H) { ++outside; continue; }
        long p = (long)fy * W + (long)fx;
        if (owner[p] >= 0) { ++dup; continue; }
        owner[p] = m;
        seed_pix[m] = (int)p;
        ++used;
    }
    free(owner);
    if (n_outside) *n_outside = outside;
    if (n_duplicate) *n_duplicate = dup;
    return used;
}

/* ------------------------------------------------------------------ */
/* geodesic Voronoi transform: multi-source Dijkstra, key (D, label)    */
/* ------------------------------------------------------------------ */
void epic_ref_voronoi(const float* C, int H, int W, const int* seed_pix,
                      int N, int conn, double* D, int* L)
{
    long HW = (long)H * W;
    int nn = conn == 4 ? 4 : 8;
    heap h = { 0, 0, 0 };
    for (long i = 0; i < HW; ++i) { D[i] = REF_INF; L[i] = -1; }
    for (int m = 0; m < N; ++m) {
        int p = seed_pix[m];
        if (p < 0) continue;
        D[p] = 0.0;
        L[p] = m;
        hpush(&h, 0.0, m, p);
    }
    while (h.n > 0) {
        hitem it = hpop(&h);
        long p = it.id;
        if (it.key != D[p] || it.tie != L[p]) continue;     /* stale */
        int px = (int)(p % W), py = (int)(p / W);
        for (int k = 0; k < nn; ++k) {
            int qx = px + NB_DX[k], qy = py + NB_DY[k];
            if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
            long q = (long)qy * W + qx;
            double cand = D[p] + step_cost(C, p, q, NB_DX[k], NB_DY[k]);
            if (cand < D[q] || (cand == D[q] && L[p] < L[q])) {
                D[q] = cand;
                L[q] = L[p];
                hpush(&h, cand, L[p], (int)q);
            }
        }
    }
    free(h.a);
}

/* single-source geodesic distance from one pixel to every pixel */
void epic_ref_geodesic_from(const float* C, int H, int W, int src_pix,
                            int conn, double* D)
{
    long HW = (long)H * W;
    int* L = (int*)malloc(sizeof(int) * HW);
    int seed = src_pix;
    epic_ref_voronoi(C, H, W, &seed, 1, conn, D, L);
    free(L);
}

/* ------------------------------------------------------------------ */
/* match graph from the Voronoi cells                                   */
/* ------------------------------------------------------------------ */
typedef struct { int m, n; double w; } etrip;

static int ecmp(const void* a, const void* b)
{
    const etrip* x = (const etrip*)a;
    const etrip* y = (const etrip*)b;
    if (x->m != y->m) return x->m < y->m ? -1 : 1;
    if (x->n != y->n) return x->n < y->n ? -1 : 1;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return 0;
}

/* Returns the number of edges (m < n, sorted by (m, n)), or -1 when more
 * than max_edges distinct edges exist. */
long epic_ref_graph(const float* C, int H, int W, const double* D,
                    const int* L, int conn, int* em, int* en, double* ew,
                    long max_edges)
{
    int nh = conn == 4 ? 2 : 4;
    long HW = (long)H * W, nt = 0, cap = 1024;
    etrip* t = (etrip*)malloc(sizeof(etrip) * cap);
    for (long p = 0; p < HW; ++p) {
        int px = (int)(p % W), py = (int)(p / W);
        for (int k = 0; k < nh; ++k) {
            int qx = px + HALF_DX[k], qy = py + HALF_DY[k];
            if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
            long q = (long)qy * W + qx;
            if (L[p] == L[q] || L[p] < 0 || L[q] < 0) continue;
            if (nt == cap) {
                cap *= 2;
                t = (etrip*)realloc(t, sizeof(etrip) * cap);
            }
            double cand = (D[p] + step_cost(C, p, q, HALF_DX[k], HALF_DY[k]))
                          + D[q];
            t[nt].m = L[p] < L[q] ? L[p] : L[q];
            t[nt].n = L[p] < L[q] ? L[q] : L[p];
            t[nt].w = cand;
            ++nt;
        }
    }
    qsort(t, (size_t)nt, sizeof(etrip), ecmp);
    long E = 0;
    for (long i = 0; i < nt; ++i) {
        if (i > 0 && t[i].m == t[i - 1].m && t[i].n == t[i - 1].n) continue;
        if (E >= max_edges) { free(t); return -1; }
        em[E] = t[i].m;
        en[E] = t[i].n;
        ew[E] = t[i].w;          /* first of a run = minimum after the sort */
        ++E;
    }
    free(t);
    return E;
}

/* ------------------------------------------------------------------ */
/* K nearest matches per match: Dijkstra on the graph                   */
/* ------------------------------------------------------------------ */
void epic_ref_knn(int N, const int* seed_pix, long E, const int* em,
                  const int* en, const double* ew, int K, int* knn_idx,
                  double* knn_d)
{
    int n_used = 0;
    for (int m = 0; m < N; ++m) n_used += seed_pix[m] >= 0;
    int Keff = K < n_used ? K : n_used;
    /* adjacency lists, both directions */
    long* rp = (long*)calloc((size_t)N + 1, sizeof(long));
    for (long e = 0; e < E; ++e) { rp[em[e] + 1]++; rp[en[e] + 1]++; }
    for (int m = 0; m < N; ++m) rp[m + 1] += rp[m];
    int* col = (int*)malloc(sizeof(int) * (size_t)(2 * E + 1));
    double* wt = (double*)malloc(sizeof(double) * (size_t)(2 * E + 1));
    long* cur = (long*)malloc(sizeof(long) * ((size_t)N + 1));
    memcpy(cur, rp, sizeof(long) * ((size_t)N + 1));
    for (long e = 0; e < E; ++e) {
        long a = cur[em[e]]++, b = cur[en[e]]++;
        col[a] = en[e]; wt[a] = ew[e];
        col[b] = em[e]; wt[b] = ew[e];
    }
    free(cur);

    #pragma omp parallel
    {
        double* dist = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
        char* done = (char*)calloc((size_t)(N > 0 ? N : 1), 1);
        int* touched = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
        for (int i = 0; i < N; ++i) dist[i] = REF_INF;
        heap h = { 0, 0, 0 };
        #pragma omp for schedule(dynamic, 16)
        for (int s = 0; s < N; ++s) {
            for (int j = 0; j < K; ++j) {
                knn_idx[(long)s * K + j] = -1;
                knn_d[(long)s * K + j] = REF_INF;
            }
            if (seed_pix[s] < 0) continue;
            int nt = 0, got = 0;
            h.n = 0;
            dist[s] = 0.0;
            touched[nt++] = s;
            hpush(&h, 0.0, s, s);
            while (h.n > 0 && got < Keff) {
                hitem it = hpop(&h);
                int u = it.id;
                if (done[u] || it.key != dist[u]) continue;
                done[u] = 1;
                knn_idx[(long)s * K + got] = u;
                knn_d[(long)s * K + got] = dist[u];
                ++got;
                for (long e = rp[u]; e < rp[u + 1]; ++e) {
                    int v = col[e];
                    if (done[v]) continue;
                    double c = dist[u] + wt[e];
                    if (c < dist[v]) {
                        if (dist[v] == REF_INF) touched[nt++] = v;
                        dist[v] = c;
                        hpush(&h, c, v, v);
                    }
                }
            }
            for (int i = 0; i < nt; ++i) { dist[touched[i]] = REF_INF; done[touched[i]] = 0; }
        }
        free(h.a);
        free(dist);
        free(done);
        free(touched);
    }
    free(rp);
    free(col);
    free(wt);
}

/* ------------------------------------------------------------------ */
/* per-match fits                                                       */
/* ------------------------------------------------------------------ */

/* Householder QR least squares for an n x 3 system with two right-hand
 * sides (columns of b, row-major n x 2).  A and b are overwritten.
 * Returns 0 on success, -1 if a diagonal entry of R is exactly zero. */
static int qr_lstsq3(double* A, double* b, int n, double* xu, double* xv)
{
    for (int k = 0; k < 3; ++k) {
        double nrm = 0.0;
        for (int i = k; i < n; ++i) nrm += A[i * 3 + k] * A[i * 3 + k];
        nrm = sqrt(nrm);
        if (nrm == 0.0) return -1;
        double alpha = A[k * 3 + k] > 0 ? -nrm : nrm;
        /* v = x - alpha e1, stored in a scratch column */
        double* v = (double*)malloc(sizeof(double) * (size_t)n);
        double vn = 0.0;
        for (int i = k; i < n; ++i) {
            v[i] = A[i * 3 + k] - (i == k ? alpha : 0.0);
            vn += v[i] * v[i];
        }
        if (vn > 0.0) {
            for (int j = k; j < 3; ++j) {
                double s = 0.0;
                for (int i = k; i < n; ++i) s += v[i] * A[i * 3 + j];
                s = 2.0 * s / vn;
                for (int i = k; i < n; ++i) A[i * 3 + j] -= s * v[i];
            }
            for (int j = 0; j < 2; ++j) {
                double s = 0.0;
                for (int i = k; i < n; ++i) s += v[i] * b[i * 2 + j];
                s = 2.0 * s / vn;
                for (int i = k; i < n; ++i) b[i * 2 + j] -= s * v[i];
            }
        }
        free(v);
    }
    double R[3][3], y[3][2];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) R[i][j] = A[i * 3 + j];
        y[i][0] = b[i * 2 + 0];
        y[i][1] = b[i * 2 + 1];
        if (R[i][i] == 0.0) return -1;
    }
    double xs[3][2];
    for (int c = 0; c < 2; ++c) {
        for (int i = 2; i >= 0; --i) {
            double s = y[i][c];
            for (int j = i + 1; j < 3; ++j) s -= R[i][j] * xs[j][c];
            xs[i][c] = s / R[i][i];
        }
    }
    xu[0] = xs[0][0]; xu[1] = xs[1][0]; xu[2] = xs[2][0];
    xv[0] = xs[0][1]; xv[1] = xs[1][1]; xv[2] = xs[2][1];
    return 0;
}

/* Weighted 2x2 covariance of the neighbour positions about their weighted
 * centroid; returns its eigenvalues (l1 >= l2).  A neighbourhood is
 * "near-collinear" when l2 <= tau * l1 (or l1 == 0). */
static void cov_eigs(const double* px, const double* py, const double* w,
                     int n, double* l1, double* l2)
{
    double sw = 0, mx = 0, my = 0;
    for (int j = 0; j < n; ++j) { sw += w[j]; mx += w[j] * px[j]; my += w[j] * py[j]; }
    mx /= sw; my /= sw;
    double sxx = 0, sxy = 0, syy = 0;
    for (int j = 0; j < n; ++j) {
        double dx = px[j] - mx, dy = py[j] - my;
        sxx += w[j] * dx * dx; sxy += w[j] * dx * dy; syy += w[j] * dy * dy;
    }
    sxx /= sw; sxy /= sw; syy /= sw;
    double tr = sxx + syy;
    double disc = sqrt((sxx - syy) * (sxx - syy) + 4.0 * sxy * sxy);
    *l1 = 0.5 * (tr + disc);
    *l2 = 0.5 * (tr - disc);
}

/* params per match: b00 b01 b10 b11 c0 c1, the displacement model
 *   u(p) = b00 (x - x_m) + b01 (y - y_m) + c0
 *   v(p) = b10 (x - x_m) + b11 (y - y_m) + c1
 * mode 0 = NW, 1 = LA; wpow = 1 or 2; status[m]: 0 LA, 1 NW by request,
 * 2 LA degenerate -> NW, -1 unused match. */
void epic_ref_fit(const float* matches, int N, const int* seed_pix,
                  const int* knn_idx, const double* knn_d, int K, double a,
                  int mode, int wpow, double deg_tau, double* params,
                  int* status)
{
    #pragma omp parallel
    {
        double* px = (double*)malloc(sizeof(double) * (size_t)K);
        double* py = (double*)malloc(sizeof(double) * (size_t)K);
        double* pu = (double*)malloc(sizeof(double) * (size_t)K);
        double* pv = (double*)malloc(sizeof(double) * (size_t)K);
        double* kw = (double*)malloc(sizeof(double) * (size_t)K);
        double* lw = (double*)malloc(sizeof(double) * (size_t)K);
        double* A = (double*)malloc(sizeof(double) * (size_t)K * 3);
        double* b = (double*)malloc(sizeof(double) * (size_t)K * 2);
        #pragma omp for schedule(dynamic, 32)
        for (int m = 0; m < N; ++m) {
            double* P = params + (long)m * 6;
            for (int i = 0; i < 6; ++i) P[i] = 0.0;
            if (seed_pix[m] < 0) { status[m] = -1; continue; }
            int n = 0;
            for (int j = 0; j < K; ++j) {
                int id = knn_idx[(long)m * K + j];
                if (id < 0) break;
                const float* r = matches + 4L * id;
                px[n] = r[0]; py[n] = r[1];
                pu[n] = (double)r[2] - (double)r[0];
                pv[n] = (double)r[3] - (double)r[1];
                kw[n] = exp(-a * knn_d[(long)m * K + j]);
                lw[n] = wpow == 1 ? kw[n] : kw[n] * kw[n];
                ++n;
            }
            /* Nadaraya-Watson, Eq. (1), on displacements */
            double sk = 0, su = 0, sv = 0;
            for (int j = 0; j < n; ++j) { sk += kw[j]; su += kw[j] * pu[j]; sv += kw[j] * pv[j]; }
            double cu = su / sk, cv = sv / sk;
            if (mode == 0) {
                P[4] = cu; P[5] = cv; status[m] = 1;
                continue;
            }
            /* locally-weighted affine, Eq. (2) */
            int degenerate = n < 3;
            if (!degenerate) {
                double l1, l2;
                cov_eigs(px, py, lw, n, &l1, &l2);
                degenerate = !(l1 > 0.0) || l2 <= deg_tau * l1;
            }
            if (!degenerate) {
                double xm = matches[4L * m + 0], ym = matches[4L * m + 1];
                for (int j = 0; j < n; ++j) {
                    double s = sqrt(lw[j]);
                    A[j * 3 + 0] = s * (px[j] - xm);
                    A[j * 3 + 1] = s * (py[j] - ym);
                    A[j * 3 + 2] = s;
                    b[j * 2 + 0] = s * pu[j];
                    b[j * 2 + 1] = s * pv[j];
                }
                double xu[3], xv[3];
                if (qr_lstsq3(A, b, n, xu, xv) == 0) {
                    P[0] = xu[0]; P[1] = xu[1]; P[4] = xu[2];
                    P[2] = xv[0]; P[3] = xv[1]; P[5] = xv[2];
                    status[m] = 0;
                    continue;
                }
            }
            P[4] = cu; P[5] = cv; status[m] = 2;
        }
        free(px); free(py); free(pu); free(pv); free(kw); free(lw); free(A); free(b);
    }
}

/* ------------------------------------------------------------------ */
/* dense assignment                                                     */
/* ------------------------------------------------------------------ */
void epic_ref_assign(int H, int W, const int* L, const float* matches,
                     const double* params, double* flow)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            long p = (long)y * W + x;
            int m = L[p];
            if (m < 0) { flow[2 * p] = flow[2 * p + 1] = NAN; continue; }
            const double* P = params + (long)m * 6;
            double dx = x - (double)matches[4L * m + 0];
            double dy = y - (double)matches[4L * m + 1];
            flow[2 * p + 0] = P[0] * dx + P[1] * dy + P[4];
            flow[2 * p + 1] = P[2] * dx + P[3] * dy + P[5];
        }
    }
}

/* ------------------------------------------------------------------ */
/* whole interpolation                                                  */
/* ------------------------------------------------------------------ */
/* stats[0..5] = used, outside, duplicate, degenerate, edges, K used.
 * Returns 0, or -3 when no match lies in the image (flow is NaN). */
int epic_ref_interp(const float* C, int H, int W, const float* matches, int N,
                    int K, double a, int mode, int conn, int wpow,
                    double deg_tau, double* flow, long* stats)
{
    long HW = (long)H * W;
    int* seed = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int outside = 0, dup = 0;
    int used = epic_ref_seeds(H, W, matches, N, seed, &outside, &dup);
    if (stats) { stats[0] = used; stats[1] = outside; stats[2] = dup; }
    if (used == 0) {
        for (long i = 0; i < 2 * HW; ++i) flow[i] = NAN;
        free(seed);
        return -3;
    }
    double* D = (double*)malloc(sizeof(double) * HW);
    int* L = (int*)malloc(sizeof(int) * HW);
    epic_ref_voronoi(C, H, W, seed, N, conn, D, L);
    long cap = 4 * HW + 1;
    int* em = (int*)malloc(sizeof(int) * cap);
    int* en = (int*)malloc(sizeof(int) * cap);
    double* ew = (double*)malloc(sizeof(double) * cap);
    long E = epic_ref_graph(C, H, W, D, L, conn, em, en, ew, cap);
    int Kc = K < used ? K : used;
    int* ki = (int*)malloc(sizeof(int) * (size_t)N * Kc);
    double* kd = (double*)malloc(sizeof(double) * (size_t)N * Kc);
    epic_ref_knn(N, seed, E, em, en, ew, Kc, ki, kd);
    double* P = (double*)malloc(sizeof(double) * (size_t)N * 6);
    int* st = (int*)malloc(sizeof(int) * (size_t)N);
    epic_ref_fit(matches, N, seed, ki, kd, Kc, a, mode, wpow, deg_tau, P, st);
    epic_ref_assign(H, W, L, matches, P, flow);
    if (stats) {
        long ndeg = 0;
        for (int m = 0; m < N; ++m) ndeg += st[m] == 2;
        stats[3] = ndeg;
        stats[4] = E;
        stats[5] = Kc;
    }
    free(seed); free(D); free(L); free(em); free(en); free(ew);
    free(ki); free(kd); free(P); free(st);
    return 0;
}

/* ------------------------------------------------------------------ */
/* consistency check of the matches (Sec. 5.1, "Pruning of matches")    */
/* ------------------------------------------------------------------ */
/* The interpolation is run once with the NW estimator (same K and a);
 * a match is kept when its own displacement u_m differs from that first
 * estimate at its pixel by at most prune_px (Euclidean norm).  At the
 * pixel of match m the NW field is the model of cell m, whose value there
 * is c_m.  Matches that are not placed on a pixel (outside the image, or
 * sharing a pixel with a lower index) are not kept.  kept[] receives the
 * original indices of the kept matches in increasing order; the count is
 * returned. */
int epic_ref_prune(const float* C, int H, int W, const float* matches, int N,
                   int K, double a, int conn, double prune_px, int* kept)
{
    long HW = (long)H * W;
    int* seed = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int outside = 0, dup = 0;
    int used = epic_ref_seeds(H, W, matches, N, seed, &outside, &dup);
    if (used == 0) { free(seed); return 0; }
    double* D = (double*)malloc(sizeof(double) * HW);
    int* L = (int*)malloc(sizeof(int) * HW);
    epic_ref_voronoi(C, H, W, seed, N, conn, D, L);
    long cap = 4 * HW + 1;
    int* em = (int*)malloc(sizeof(int) * cap);
    int* en = (int*)malloc(sizeof(int) * cap);
    double* ew = (double*)malloc(sizeof(double) * cap);
    long E = epic_ref_graph(C, H, W, D, L, conn, em, en, ew, cap);
    int Kc = K < used ? K : used;
    int* ki = (int*)malloc(sizeof(int) * (size_t)N * Kc);
    double* kd = (double*)malloc(sizeof(double) * (size_t)N * Kc);
    epic_ref_knn(N, seed, E, em, en, ew, Kc, ki, kd);
    double* P = (double*)malloc(sizeof(double) * (size_t)N * 6);
    int* st = (int*)malloc(sizeof(int) * (size_t)N);
    epic_ref_fit(matches, N, seed, ki, kd, Kc, a, 0, 2, 0.0, P, st);
    int nk = 0;
    for (int m = 0; m < N; ++m) {
        if (seed[m] < 0) continue;
        double du = ((double)matches[4L * m + 2] - matches[4L * m + 0]) - P[6L * m + 4];
        double dv = ((double)matches[4L * m + 3] - matches[4L * m + 1]) - P[6L * m + 5];
        if (sqrt(du * du + dv * dv) <= prune_px) kept[nk++] = m;
    }
    free(seed); free(D); free(L); free(em); free(en); free(ew);
    free(ki); free(kd); free(P); free(st);
    return nk;
}

/* ------------------------------------------------------------------ */
/* cost map from the image gradient (Table 2, contour row: the norm of  */
/* the image gradient; the same norm sets the smoothness weight, Sec. 4) */
/* ------------------------------------------------------------------ */
/* C(p) = sqrt(sum over channels of gx^2 + gy^2) + eps, with central
 * differences gx = (I(x+1) - I(x-1)) / 2, gy = (I(y+1) - I(y-1)) / 2 and
 * the border pixel repeated outside the image.  image: H*W*ch float,
 * channels interleaved. */
void epic_ref_grad_cost(const float* image, int H, int W, int ch, double eps, double* cost)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        int yu = y > 0 ? y - 1 : 0, yd = y < H - 1 ? y + 1 : H - 1;
        for (int x = 0; x < W; ++x) {
            int xl = x > 0 ? x - 1 : 0, xr = x < W - 1 ? x + 1 : W - 1;
            double s = 0.0;
            for (int c = 0; c < ch; ++c) {
                double gx = ((double)image[((long)y * W + xr) * ch + c] -
                             (double)image[((long)y * W + xl) * ch + c]) / 2.0;
                double gy = ((double)image[((long)yd * W + x) * ch + c] -
                             (double)image[((long)yu * W + x) * ch + c]) / 2.0;
                s += gx * gx + gy * gy;
            }
            cost[(long)y * W + x] = sqrt(s) + eps;
        }
    }
}

/* ------------------------------------------------------------------ */
/* exact per-pixel geodesic interpolation (Table 2, "Geodesic (exact)") */
/* ------------------------------------------------------------------ */
typedef struct { double d; int m; } dm_pair;

static int dm_cmp(const void* a, const void* b)
{
    const dm_pair* x = (const dm_pair*)a;
    const dm_pair* y = (const dm_pair*)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->m > y->m) - (x->m < y->m);
}

/* The variant without the approximation of Sec. 3.4: every pixel p gets its
 * own K nearest matches under the discretised geodesic distance of Eq. (3)
 * itself, D_G(p, p_m) -- one Dijkstra from p over the pixel graph --
 * ordered by (distance, index), weights exp(-a D_G), and its own NW
 * (Eq. 1) or LA (Eq. 2) estimate, evaluated at p (the displacement at p of
 * the affine map fitted about p).  Matches are placed, dropped and
 * deduplicated as in epic_ref_seeds; K is clamped to the placed matches;
 * the near-collinear LA test and its NW fallback are those of epic_ref_fit.
 * pix[0..npix): the pixels (y*W + x) to evaluate; flow, knn_idx, knn_d
 * receive npix rows (knn outputs may be NULL).  Returns 0, or -3 when no
 * match lies in the image (flow NaN). */
int epic_ref_exact(const float* C, int H, int W, const float* matches, int N,
                   int K, double a, int mode, int conn, int wpow, double deg_tau,
                   const long* pix, long npix, double* flow, int* knn_idx, double* knn_d)
{
    long HW = (long)H * W;
    int* seed = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int outside = 0, dup = 0;
    int used = epic_ref_seeds(H, W, matches, N, seed, &outside, &dup);
    if (used == 0) {
        for (long i = 0; i < 2 * npix; ++i) flow[i] = NAN;
        free(seed);
        return -3;
    }
    int Kc = K < used ? K : used;
    #pragma omp parallel
    {
        double* D = (double*)malloc(sizeof(double) * HW);
        dm_pair* cand = (dm_pair*)malloc(sizeof(dm_pair) * (size_t)used);
        double* px = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* py = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* pu = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* pv = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* kw = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* lw = (double*)malloc(sizeof(double) * (size_t)Kc);
        double* A = (double*)malloc(sizeof(double) * (size_t)Kc * 3);
        double* b = (double*)malloc(sizeof(double) * (size_t)Kc * 2);
        #pragma omp for schedule(dynamic, 1)
        for (long t = 0; t < npix; ++t) {
            long p = pix[t];
            double xp = (double)(p % W), yp = (double)(p / W);
            epic_ref_geodesic_from(C, H, W, (int)p, conn, D);
            int nc = 0;
            for (int m = 0; m < N; ++m)
                if (seed[m] >= 0) { cand[nc].d = D[seed[m]]; cand[nc].m = m; ++nc; }
            qsort(cand, (size_t)nc, sizeof(dm_pair), dm_cmp);
            for (int j = 0; j < Kc; ++j) {
                const float* r = matches + 4L * cand[j].m;
                px[j] = r[0]; py[j] = r[1];
                pu[j] = (double)r[2] - (double)r[0];
                pv[j] = (double)r[3] - (double)r[1];
                kw[j] = exp(-a * cand[j].d);
                lw[j] = wpow == 1 ? kw[j] : kw[j] * kw[j];
                if (knn_idx) knn_idx[t * K + j] = cand[j].m;
                if (knn_d) knn_d[t * K + j] = cand[j].d;
            }
            for (int j = Kc; j < K; ++j) {
                if (knn_idx) knn_idx[t * K + j] = -1;
                if (knn_d) knn_d[t * K + j] = REF_INF;
            }
            /* Nadaraya-Watson, Eq. (1), on displacements */
            double sk = 0, su = 0, sv = 0;
            for (int j = 0; j < Kc; ++j) { sk += kw[j]; su += kw[j] * pu[j]; sv += kw[j] * pv[j]; }
            double fu = su / sk, fv = sv / sk;
            if (mode == 1) {
                /* LA, Eq. (2), about the pixel itself: rows k [x - x_p, y - y_p, 1] */
                int degenerate = Kc < 3;
                if (!degenerate) {
                    double l1, l2;
                    cov_eigs(px, py, lw, Kc, &l1, &l2);
                    degenerate = !(l1 > 0.0) || l2 <= deg_tau * l1;
                }
                if (!degenerate) {
                    for (int j = 0; j < Kc; ++j) {
                        double s = sqrt(lw[j]);
                        A[j * 3 + 0] = s * (px[j] - xp);
                        A[j * 3 + 1] = s * (py[j] - yp);
                        A[j * 3 + 2] = s;
                        b[j * 2 + 0] = s * pu[j];
                        b[j * 2 + 1] = s * pv[j];
                    }
                    double xu[3], xv[3];
                    if (qr_lstsq3(A, b, Kc, xu, xv) == 0) { fu = xu[2]; fv = xv[2]; }
                }
            }
            flow[2 * t + 0] = fu;
            flow[2 * t + 1] = fv;
        }
        free(D); free(cand); free(px); free(py); free(pu); free(pv); free(kw); free(lw); free(A); free(b);
    }
    free(seed);
    return 0;
}
