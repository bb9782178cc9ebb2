/*
 * slfo — plain FP64 CPU oracle of the superpixel-plane matching cost.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Independent of
 * the HIP library (no shared code, headers or tables).
 *
 * Written from Chuchvara, Barsi, Gotchev, "Fast and Accurate Depth Estimation
 * from Sparse Light Fields": superpixels (Sec. III-A), partly randomised
 * plane sweep with TSSD (Sec. III-B, eqs. 1-2), iterative refinement with
 * propagation kernel, triangle normals and the energy E = E_c E_s (Sec.
 * III-C, eqs. 3-11), Jacobi ping-pong over all superpixels of all views
 * (Sec. III-E).  Everything is FP64; sums run in a fixed order (neighbour
 * views in list order, pixels in raster order), and superpixels are
 * independent, so results do not depend on the OpenMP thread count.
 * Build with -ffp-contract=off.
 */
#include "slfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct slfo_ctx {
    slfo_rig rig;
    slfo_params p;
    int V;
    int64_t *sp_off;   /* [V+1] */
    int64_t S;         /* total superpixels */
    int32_t *area;     /* [S] */
    double *cen;       /* [S][2] */
    double *col;       /* [S][3] */
    int64_t *px_off;   /* [S+1] into px */
    int32_t *px;       /* pixel index u + W v inside its view, raster order per superpixel */
    double *Kinv;      /* [V][9] */
};

/* ring of the eight grid neighbours, gy pointing down; consecutive entries are adjacent */
static const int RING_DX[8] = {1, 1, 0, -1, -1, -1, 0, 1};
static const int RING_DY[8] = {0, 1, 1, 1, 0, -1, -1, -1};

/* ---------------------------------------------------------------- helpers */

static void inv3(const double *m, double *o)
{
    double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5], g = m[6], h = m[7], i = m[8];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double det = a * A + b * B + c * C;
    o[0] = A / det;
    o[1] = -(b * i - c * h) / det;
    o[2] = (b * f - c * e) / det;
    o[3] = B / det;
    o[4] = (a * i - c * g) / det;
    o[5] = -(a * f - c * d) / det;
    o[6] = C / det;
    o[7] = -(a * h - b * g) / det;
    o[8] = (a * e - b * d) / det;
}

static void matmul3(const double *a, const double *b, double *o)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) o[3 * r + c] = a[3 * r] * b[c] + a[3 * r + 1] * b[3 + c] + a[3 * r + 2] * b[6 + c];
}

static void matvec3(const double *a, const double *x, double *o)
{
    for (int r = 0; r < 3; ++r) o[r] = a[3 * r] * x[0] + a[3 * r + 1] * x[1] + a[3 * r + 2] * x[2];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static int W_of(const slfo_ctx *c, int v) { return c->rig.width[v]; }
static int H_of(const slfo_ctx *c, int v) { return c->rig.height[v]; }

static const uint8_t *rgb_of(const slfo_ctx *c, int v) { return c->rig.rgb + 3 * c->rig.pix_off[v]; }
static const int32_t *lab_of(const slfo_ctx *c, int v) { return c->rig.labels + c->rig.pix_off[v]; }

/* K_v^-1 (u, v, 1)^T: the viewing ray with unit z */
static void backproject(const slfo_ctx *c, int v, double u, double vv, double *ray)
{
    double p[3] = {u, vv, 1.0};
    matvec3(c->Kinv + 9 * v, p, ray);
}

/* relative pose of camera i with respect to camera r: R_ri = R_i R_r^T, t_ri = t_i - R_ri t_r */
static void rel_pose(const slfo_ctx *c, int r, int i, double *Rri, double *tri)
{
    const double *Rr = c->rig.R + 9 * r, *Ri = c->rig.R + 9 * i;
    double RrT[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) RrT[3 * a + b] = Rr[3 * b + a];
    matmul3(Ri, RrT, Rri);
    double Rt[3];
    matvec3(Rri, c->rig.t + 3 * r, Rt);
    for (int a = 0; a < 3; ++a) tri[a] = c->rig.t[3 * i + a] - Rt[a];
}

/* plane-induced homography (Sec. III-B): H = K_i (R_ri + t_ri n^T / delta) K_r^-1 */
static void homography(const slfo_ctx *c, int r, int i, const double *n, double delta, double *H)
{
    double Rri[9], tri[3], M[9], T[9];
    rel_pose(c, r, i, Rri, tri);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = Rri[3 * a + b] + tri[a] * n[b] / delta;
    matmul3(c->rig.K + 9 * i, M, T);
    matmul3(T, c->Kinv + 9 * r, H);
}

/* colour similarity weight, eq. (7), squared Euclidean RGB distance */
static double omega(const slfo_ctx *c, const double *ca, const double *cb)
{
    double d0 = ca[0] - cb[0], d1 = ca[1] - cb[1], d2 = ca[2] - cb[2];
    double a = c->p.alpha;
    return exp(-(d0 * d0 + d1 * d1 + d2 * d2) / (2.0 * a * a));
}

static int64_t gid(const slfo_ctx *c, int v, int s) { return c->sp_off[v] + s; }

/* cell s + (dx, dy) of view v, or -1 if outside the grid or empty */
static int cell_at(const slfo_ctx *c, int v, int s, int dx, int dy)
{
    int gw = c->rig.grid_w[v], gh = c->rig.grid_h[v];
    int gx = s % gw + dx, gy = s / gw + dy;
    if (gx < 0 || gx >= gw || gy < 0 || gy >= gh) return -1;
    int k = gy * gw + gx;
    return c->area[gid(c, v, k)] > 0 ? k : -1;
}

/* 3D plane (n, delta) of a stored plane (d, n) of superpixel s in view v */
static double plane_delta(const slfo_ctx *c, int v, int s, const double *pl)
{
    const double *cs = c->cen + 2 * gid(c, v, s);
    double ray[3];
    backproject(c, v, cs[0], cs[1], ray);
    return pl[0] * dot3(pl + 1, ray);
}

/* ------------------------------------------------------------ public misc */

/* SplitMix64 output function (Steele, Lea, Flood 2014; Stafford's mix 13) */
uint64_t slfo_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void slfo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int params_ok(const slfo_params *p)
{
    if (p->levels < 1) return 0;
    if (!(p->d_min > 0) || !(p->d_max > p->d_min) || !isfinite(p->d_max)) return 0;
    if (!(p->tssd_T > 0) || !(p->sigma > 0) || !(p->alpha > 0)) return 0;
    if (p->kernel_step < 1) return 0;
    return 1;
}

slfo_ctx *slfo_create(const slfo_rig *rig, const slfo_params *p, int *err)
{
    *err = -1;
    if (!rig || !p || rig->n_views < 1 || !params_ok(p)) return NULL;
    int V = rig->n_views;
    for (int v = 0; v < V; ++v) {
        if (rig->width[v] < 2 || rig->height[v] < 2 || rig->grid_w[v] < 1 || rig->grid_h[v] < 1) return NULL;
        for (int j = rig->nbr_off[v]; j < rig->nbr_off[v + 1]; ++j)
            if (rig->nbr[j] < 0 || rig->nbr[j] >= V || rig->nbr[j] == v) return NULL;
        if (rig->nbr_off[v + 1] <= rig->nbr_off[v]) return NULL;
    }
    slfo_ctx *c = (slfo_ctx *)calloc(1, sizeof(slfo_ctx));
    if (!c) {
        *err = -3;
        return NULL;
    }
    c->rig = *rig;
    c->p = *p;
    c->V = V;
    c->sp_off = (int64_t *)malloc(sizeof(int64_t) * (V + 1));
    c->Kinv = (double *)malloc(sizeof(double) * 9 * V);
    c->sp_off[0] = 0;
    for (int v = 0; v < V; ++v) {
        c->sp_off[v + 1] = c->sp_off[v] + (int64_t)rig->grid_w[v] * rig->grid_h[v];
        inv3(rig->K + 9 * v, c->Kinv + 9 * v);
    }
    c->S = c->sp_off[V];
    int64_t npx = rig->pix_off[V];
    c->area = (int32_t *)calloc(c->S, sizeof(int32_t));
    c->cen = (double *)calloc(2 * c->S, sizeof(double));
    c->col = (double *)calloc(3 * c->S, sizeof(double));
    c->px_off = (int64_t *)calloc(c->S + 1, sizeof(int64_t));
    c->px = (int32_t *)malloc(sizeof(int32_t) * (npx > 0 ? npx : 1));
    if (!c->area || !c->cen || !c->col || !c->px_off || !c->px) {
        slfo_destroy(c);
        *err = -3;
        return NULL;
    }
    /* Superpixel statistics (Sec. III-A, III-C-1): area, centroid, mean colour */
    for (int v = 0; v < V; ++v) {
        int W = rig->width[v], H = rig->height[v];
        int64_t K = (int64_t)rig->grid_w[v] * rig->grid_h[v];
        const int32_t *lab = lab_of(c, v);
        const uint8_t *img = rgb_of(c, v);
        for (int64_t i = 0; i < (int64_t)W * H; ++i) {
            if (lab[i] < 0 || lab[i] >= K) {
                slfo_destroy(c);
                *err = -2;
                return NULL;
            }
            c->area[gid(c, v, lab[i])]++;
        }
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t i = (int64_t)y * W + x;
                int64_t g = gid(c, v, lab[i]);
                c->cen[2 * g] += x;
                c->cen[2 * g + 1] += y;
                for (int ch = 0; ch < 3; ++ch) c->col[3 * g + ch] += img[3 * i + ch] / 255.0;
            }
    }
    for (int64_t g = 0; g < c->S; ++g) {
        c->px_off[g + 1] = c->px_off[g] + c->area[g];
        if (c->area[g] > 0) {
            c->cen[2 * g] /= c->area[g];
            c->cen[2 * g + 1] /= c->area[g];
            for (int ch = 0; ch < 3; ++ch) c->col[3 * g + ch] /= c->area[g];
        }
    }
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (c->S > 0 ? c->S : 1));
    memcpy(fill, c->px_off, sizeof(int64_t) * c->S);
    for (int v = 0; v < V; ++v) {
        int W = rig->width[v], H = rig->height[v];
        const int32_t *lab = lab_of(c, v);
        for (int64_t i = 0; i < (int64_t)W * H; ++i) {
            int64_t g = gid(c, v, lab[i]);
            c->px[fill[g]++] = (int32_t)i;
        }
    }
    free(fill);
    *err = 0;
    return c;
}

void slfo_destroy(slfo_ctx *c)
{
    if (!c) return;
    free(c->sp_off);
    free(c->area);
    free(c->cen);
    free(c->col);
    free(c->px_off);
    free(c->px);
    free(c->Kinv);
    free(c);
}

int slfo_set_params(slfo_ctx *c, const slfo_params *p)
{
    if (!params_ok(p)) return -1;
    c->p = *p;
    return 0;
}

int64_t slfo_sp_offset(const slfo_ctx *c, int view) { return c->sp_off[view]; }
int64_t slfo_sp_total(const slfo_ctx *c) { return c->S; }

int slfo_sp_stats(const slfo_ctx *c, int32_t *area, double *centroid, double *colour)
{
    if (area) memcpy(area, c->area, sizeof(int32_t) * c->S);
    if (centroid) memcpy(centroid, c->cen, sizeof(double) * 2 * c->S);
    if (colour) memcpy(colour, c->col, sizeof(double) * 3 * c->S);
    return 0;
}

int slfo_homography(const slfo_ctx *c, int r, int i, const double n[3], double delta, double H[9])
{
    if (r < 0 || r >= c->V || i < 0 || i >= c->V) return -1;
    homography(c, r, i, n, delta, H);
    return 0;
}

/* --------------------------------------------------------------- sweep */

/* Inverse-depth level k of superpixel s in view r (Sec. III-B): L bins of
 * width Delta over [1/d_max, 1/d_min]; with jitter, a per-superpixel uniform
 * offset u in [0, 1) of one bin, u = top 24 bits of mix64(key) / 2^24. */
double slfo_level_q(const slfo_ctx *c, int r, int s, int k)
{
    double qmin = 1.0 / c->p.d_max, qmax = 1.0 / c->p.d_min;
    double delta = (qmax - qmin) / c->p.levels;
    double u = 0.0;
    if (c->p.jitter) {
        uint64_t key = c->p.seed ^ ((uint64_t)r << 48) ^ ((uint64_t)s << 24) ^ (uint64_t)k;
        u = (double)(slfo_mix64(key) >> 40) * (1.0 / 16777216.0);
    }
    return qmin + (k + u) * delta;
}

/* bilinear sample of view i at (x, y), integer pixel centres, taps clamped so
 * x0 <= W-2 (the caller guarantees 0 <= x <= W-1, 0 <= y <= H-1) */
static void bilinear(const slfo_ctx *c, int i, double x, double y, double *out)
{
    int W = W_of(c, i), H = H_of(c, i);
    int x0 = (int)floor(x), y0 = (int)floor(y);
    if (x0 > W - 2) x0 = W - 2;
    if (y0 > H - 2) y0 = H - 2;
    double fx = x - x0, fy = y - y0;
    const uint8_t *img = rgb_of(c, i);
    const uint8_t *p00 = img + 3 * ((int64_t)y0 * W + x0);
    const uint8_t *p10 = p00 + 3;
    const uint8_t *p01 = p00 + 3 * (int64_t)W;
    const uint8_t *p11 = p01 + 3;
    for (int ch = 0; ch < 3; ++ch) {
        double top = (1.0 - fx) * (p00[ch] / 255.0) + fx * (p10[ch] / 255.0);
        double bot = (1.0 - fx) * (p01[ch] / 255.0) + fx * (p11[ch] / 255.0);
        out[ch] = (1.0 - fy) * top + fy * bot;
    }
}

/* Eq. (2) inner sums: sum over neighbour views i and pixels p of TSSD (eq. 1)
 * for plane (n, delta).  A sample that lands behind camera i or outside its
 * image costs T. */
static double tssd_sum(const slfo_ctx *c, int r, int s, const double *n, double delta)
{
    int64_t g = gid(c, r, s);
    int Wr = W_of(c, r);
    const uint8_t *ref = rgb_of(c, r);
    double T = c->p.tssd_T;
    double total = 0.0;
    for (int j = c->rig.nbr_off[r]; j < c->rig.nbr_off[r + 1]; ++j) {
        int i = c->rig.nbr[j];
        double H[9];
        homography(c, r, i, n, delta, H);
        int Wi = W_of(c, i), Hi = H_of(c, i);
        for (int64_t q = c->px_off[g]; q < c->px_off[g + 1]; ++q) {
            int pix = c->px[q];
            double pu = pix % Wr, pv = pix / Wr;
            double hp[3] = {H[0] * pu + H[1] * pv + H[2], H[3] * pu + H[4] * pv + H[5], H[6] * pu + H[7] * pv + H[8]};
            double e = T;
            if (hp[2] > 0.0) {
                double x = hp[0] / hp[2], y = hp[1] / hp[2];
                if (x >= 0.0 && x <= Wi - 1 && y >= 0.0 && y <= Hi - 1) {
                    double b[3];
                    bilinear(c, i, x, y, b);
                    double ssd = 0.0;
                    for (int ch = 0; ch < 3; ++ch) {
                        double d = ref[3 * pix + ch] / 255.0 - b[ch];
                        ssd += d * d;
                    }
                    e = ssd < T ? ssd : T;
                }
            }
            total += e;
        }
    }
    return total;
}

static int n_nbr(const slfo_ctx *c, int r) { return c->rig.nbr_off[r + 1] - c->rig.nbr_off[r]; }

static double norm_cost(const slfo_ctx *c, int r, int s, double C)
{
    return C / ((double)c->area[gid(c, r, s)] * n_nbr(c, r) * c->p.tssd_T);
}

double slfo_sweep_cost_plane(const slfo_ctx *c, int r, int s, const double plane[4])
{
    if (r < 0 || r >= c->V || s < 0 || s >= c->sp_off[r + 1] - c->sp_off[r]) return NAN;
    if (c->area[gid(c, r, s)] == 0) return NAN;
    double delta = plane_delta(c, r, s, plane);
    return norm_cost(c, r, s, tssd_sum(c, r, s, plane + 1, delta));
}

int slfo_sweep_sp(const slfo_ctx *c, int r, int s, double plane[4], double *cost, int32_t *choice, double *margin)
{
    if (r < 0 || r >= c->V || s < 0 || s >= c->sp_off[r + 1] - c->sp_off[r]) return -1;
    if (c->area[gid(c, r, s)] == 0) {
        plane[0] = plane[1] = plane[2] = plane[3] = 0.0;
        *cost = 0.0;
        *choice = -1;
        *margin = 0.0;
        return 0;
    }
    static const double front[3] = {0.0, 0.0, 1.0}; /* fronto-parallel in camera r */
    double best = INFINITY, second = INFINITY;
    int kb = -1;
    for (int k = 0; k < c->p.levels; ++k) {
        double d = 1.0 / slfo_level_q(c, r, s, k);
        /* n = (0,0,1): delta = d (n . K^-1 c~) = d because the ray has unit z */
        double cb = norm_cost(c, r, s, tssd_sum(c, r, s, front, d));
        if (cb < best) {
            second = best;
            best = cb;
            kb = k;
        } else if (cb < second) {
            second = cb;
        }
    }
    plane[0] = 1.0 / slfo_level_q(c, r, s, kb);
    plane[1] = 0.0;
    plane[2] = 0.0;
    plane[3] = 1.0;
    *cost = best;
    *choice = kb;
    *margin = second - best;
    return 0;
}

int slfo_sweep_all(const slfo_ctx *c, double *planes, double *cost, int32_t *choice, double *margin)
{
    int64_t S = c->S;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t g = 0; g < S; ++g) {
        int v = 0;
        while (g >= c->sp_off[v + 1]) ++v;
        bad |= slfo_sweep_sp(c, v, (int)(g - c->sp_off[v]), planes + 4 * g, cost + g, choice + g, margin + g) != 0;
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------- energy */

/* Smoothness, eqs. (5)-(7): colour-weighted mean over the non-empty grid
 * neighbours j of a Gaussian agreement between j's centroid depth in A and
 * this plane extrapolated to j's centroid (0 if the plane is behind the
 * camera there).  1 when there are no neighbours. */
static double e_smooth(const slfo_ctx *c, const double *A, int r, int s, const double *n, double delta)
{
    int64_t g = gid(c, r, s);
    double sw = 0.0, sws = 0.0;
    int M = 0;
    for (int j = 0; j < 8; ++j) {
        int k = cell_at(c, r, s, RING_DX[j], RING_DY[j]);
        if (k < 0) continue;
        int64_t gk = gid(c, r, k);
        ++M;
        double w = omega(c, c->col + 3 * g, c->col + 3 * gk);
        double ray[3];
        backproject(c, r, c->cen[2 * gk], c->cen[2 * gk + 1], ray);
        double tt = dot3(n, ray);
        double sj = 0.0;
        if (tt > 0.0) {
            double dhat = delta / tt;
            double dd = A[4 * gk] - dhat;
            sj = exp(-dd * dd / (2.0 * c->p.sigma * c->p.sigma));
        }
        sw += w;
        sws += w * sj;
    }
    if (M == 0) return 1.0;
    return sws / sw;
}

/* min over the non-empty grid neighbours of omega(C_s, C_j); 1 without neighbours (eq. 11) */
static double omega_min(const slfo_ctx *c, int r, int s)
{
    int64_t g = gid(c, r, s);
    double m = 1.0;
    for (int j = 0; j < 8; ++j) {
        int k = cell_at(c, r, s, RING_DX[j], RING_DY[j]);
        if (k < 0) continue;
        double w = omega(c, c->col + 3 * g, c->col + 3 * gid(c, r, k));
        if (w < m) m = w;
    }
    return m;
}

/* Consistency, eqs. (8)-(11).  For each neighbour view i and pixel p of s:
 * D = depth of p on the plane, (x, y, w) = H_i p~, z = D w is the depth of
 * the 3D point in camera i; the nearest pixel of view i gives the superpixel
 * l whose colour enters S_i (eq. 9) and whose plane in A gives D(p^i) at the
 * continuous projection.  z <= D(p^i) (1 + tau) counts into X (eq. 10),
 * otherwise into Y (eq. 11).  Pixels that land behind a camera or outside
 * view i are unseen: they add nothing to S_i's sum (whose denominator stays
 * |Omega|) and join neither X nor Y. */
static double e_consist(const slfo_ctx *c, const double *A, int r, int s, const double *n, double delta)
{
    int64_t g = gid(c, r, s);
    int Wr = W_of(c, r);
    double area = c->area[g];
    const double *Cs = c->col + 3 * g;
    double wmin = omega_min(c, r, s);
    double sig2 = 2.0 * c->p.sigma * c->p.sigma;
    double sum = 0.0;
    for (int j = c->rig.nbr_off[r]; j < c->rig.nbr_off[r + 1]; ++j) {
        int i = c->rig.nbr[j];
        double H[9];
        homography(c, r, i, n, delta, H);
        int Wi = W_of(c, i), Hi = H_of(c, i);
        const int32_t *lab_i = lab_of(c, i);
        double s_omega = 0.0, gX = 0.0;
        int64_t nX = 0;
        int anyY = 0;
        for (int64_t q = c->px_off[g]; q < c->px_off[g + 1]; ++q) {
            int pix = c->px[q];
            double pu = pix % Wr, pv = pix / Wr;
            double ray[3];
            backproject(c, r, pu, pv, ray);
            double iota = dot3(n, ray) / delta; /* inverse depth of p on the plane */
            if (!(iota > 0.0)) continue;
            double D = 1.0 / iota;
            double hp[3] = {H[0] * pu + H[1] * pv + H[2], H[3] * pu + H[4] * pv + H[5], H[6] * pu + H[7] * pv + H[8]};
            if (!(hp[2] > 0.0)) continue;
            double z = D * hp[2];
            double x = hp[0] / hp[2], y = hp[1] / hp[2];
            double ui = floor(x + 0.5), vi = floor(y + 0.5);
            if (ui < 0.0 || ui > Wi - 1 || vi < 0.0 || vi > Hi - 1) continue;
            int l = lab_i[(int64_t)vi * Wi + (int64_t)ui];
            int64_t gl = gid(c, i, l);
            s_omega += omega(c, Cs, c->col + 3 * gl);
            /* D(p^i): plane of (i, l) in A at the continuous projection (x, y) */
            const double *pl = A + 4 * gl;
            double dl = plane_delta(c, i, l, pl);
            double rayi[3];
            backproject(c, i, x, y, rayi);
            double inv = dot3(pl + 1, rayi) / dl;
            double Di = inv > 0.0 ? 1.0 / inv : INFINITY;
            if (z <= Di * (1.0 + c->p.occ_tol)) {
                ++nX;
                if (isfinite(Di)) {
                    double dz = z - Di;
                    gX += exp(-dz * dz / sig2);
                }
            } else {
                anyY = 1;
            }
        }
        double Si = s_omega / area;
        double Vi = nX > 0 ? Si * gX / (double)nX : 0.0;
        double Oi = (anyY && (c->p.term_mask & 4u)) ? c->p.eta * (1.0 - wmin) : 0.0;
        sum += Vi + Oi;
    }
    return sum / n_nbr(c, r);
}

/* E = E_c E_s (eq. 3) of the 3D plane (n, delta) for superpixel s of view r */
static double energy_nd(const slfo_ctx *c, const double *A, int r, int s, const double *n, double delta)
{
    if (c->p.energy_mode == 1) return -norm_cost(c, r, s, tssd_sum(c, r, s, n, delta));
    double Es = (c->p.term_mask & 1u) ? e_smooth(c, A, r, s, n, delta) : 1.0;
    double Ec = (c->p.term_mask & 2u) ? e_consist(c, A, r, s, n, delta) : 1.0;
    return Ec * Es;
}

/* Parity instrument, not part of the method.  The consistency term takes two
 * discrete decisions per sample: the nearest pixel of view i (eq. 9, round
 * half up, which also decides whether the sample is inside view i) and the
 * visible / occluded split (eqs. 10-11).  An implementation that forms x, y
 * or z in lower precision may take either side of a decision whose value lies
 * within its rounding of the threshold.  This returns an upper bound of how
 * much E (eq. 3) can change when any such decisions flip: per view, k samples
 * within eps_px of a rounding threshold or within eps_rel (relative) of the
 * split change S_i by at most k / |Omega| (omega in [0, 1]) and the mean of
 * the X samples' Gaussians by at most k / max(|X| - k, 1), so V_i by at most
 * their sum; O_i can toggle if |Y| <= k; E_c averages the views and E
 * multiplies E_s.  Returns 0 when no decision is that close. */
double slfo_energy_flip_bound(const slfo_ctx *c, const double *A, int r, int s, const double plane[4], double eps_px,
                              double eps_rel)
{
    if (r < 0 || r >= c->V || s < 0 || s >= c->sp_off[r + 1] - c->sp_off[r]) return NAN;
    int64_t g = gid(c, r, s);
    if (c->area[g] == 0 || c->p.energy_mode == 1 || !(c->p.term_mask & 2u)) return 0.0;
    const double *n = plane + 1;
    double delta = plane_delta(c, r, s, plane);
    int Wr = W_of(c, r);
    double area = c->area[g];
    double wmin = omega_min(c, r, s);
    double total = 0.0;
    for (int j = c->rig.nbr_off[r]; j < c->rig.nbr_off[r + 1]; ++j) {
        int i = c->rig.nbr[j];
        double H[9];
        homography(c, r, i, n, delta, H);
        int Wi = W_of(c, i), Hi = H_of(c, i);
        const int32_t *lab_i = lab_of(c, i);
        int64_t nX = 0, nY = 0, k = 0;
        for (int64_t q = c->px_off[g]; q < c->px_off[g + 1]; ++q) {
            int pix = c->px[q];
            double pu = pix % Wr, pv = pix / Wr;
            double ray[3];
            backproject(c, r, pu, pv, ray);
            double iota = dot3(n, ray) / delta;
            if (!(iota > 0.0)) continue;
            double D = 1.0 / iota;
            double hp[3] = {H[0] * pu + H[1] * pv + H[2], H[3] * pu + H[4] * pv + H[5], H[6] * pu + H[7] * pv + H[8]};
            if (!(hp[2] > 0.0)) continue;
            double z = D * hp[2];
            double x = hp[0] / hp[2], y = hp[1] / hp[2];
            double fx = x + 0.5 - floor(x + 0.5), fy = y + 0.5 - floor(y + 0.5);
            int near = fx < eps_px || fx > 1.0 - eps_px || fy < eps_px || fy > 1.0 - eps_px;
            double ui = floor(x + 0.5), vi = floor(y + 0.5);
            if (ui < 0.0 || ui > Wi - 1 || vi < 0.0 || vi > Hi - 1) {
                k += near;
                continue;
            }
            int l = lab_i[(int64_t)vi * Wi + (int64_t)ui];
            int64_t gl = gid(c, i, l);
            const double *pl = A + 4 * gl;
            double dl = plane_delta(c, i, l, pl);
            double rayi[3];
            backproject(c, i, x, y, rayi);
            double inv = dot3(pl + 1, rayi) / dl;
            double Di = inv > 0.0 ? 1.0 / inv : INFINITY;
            double lim = Di * (1.0 + c->p.occ_tol);
            if (z <= lim) ++nX; else ++nY;
            if (isfinite(lim) && fabs(z - lim) <= eps_rel * z) near = 1;
            k += near;
        }
        if (k == 0) continue;
        double b = (double)k / area + (double)k / (double)(nX - k > 1 ? nX - k : 1);
        if (b > 1.0) b = 1.0;   /* V_i lies in [0, 1] */
        if ((c->p.term_mask & 4u) && nY <= k) b += c->p.eta * (1.0 - wmin);
        total += b;
    }
    double Es = (c->p.term_mask & 1u) ? e_smooth(c, A, r, s, n, delta) : 1.0;
    return Es * total / n_nbr(c, r);
}

double slfo_energy(const slfo_ctx *c, const double *A, int r, int s, const double plane[4])
{
    if (r < 0 || r >= c->V || s < 0 || s >= c->sp_off[r + 1] - c->sp_off[r]) return NAN;
    if (c->area[gid(c, r, s)] == 0) return NAN;
    return energy_nd(c, A, r, s, plane + 1, plane_delta(c, r, s, plane));
}

/* ---------------------------------------------------------- refinement */

int slfo_kernel_radius(const slfo_ctx *c, int r, int iter)
{
    int R0 = c->p.kernel_radius_init;
    if (R0 <= 0) {
        double S = sqrt((double)W_of(c, r) * H_of(c, r) / ((double)c->rig.grid_w[r] * c->rig.grid_h[r]));
        int m = W_of(c, r) < H_of(c, r) ? W_of(c, r) : H_of(c, r);
        R0 = (int)floor(m / (2.0 * S));
    }
    return iter >= 1 ? R0 / iter : R0;
}

typedef struct {
    int32_t *slots;
    double *planes, *energies;
    int cap, n;
} trace_t;

typedef struct {
    double best_E, second_E;
    double best_plane[4];
    int best_slot;
    int evaluated;
    trace_t *tr;
} argmax_t;

/* evaluate candidate (n, delta) as slot `slot`; replace the best only on strict improvement */
static void consider(const slfo_ctx *c, const double *A, int r, int s, const double *n, double delta, int slot,
                     argmax_t *st)
{
    double ray[3];
    const double *cs = c->cen + 2 * gid(c, r, s);
    backproject(c, r, cs[0], cs[1], ray);
    double tt = dot3(n, ray);
    if (!(tt > 0.0) || !(delta > 0.0)) return; /* not in front of camera r at this centroid */
    double E = energy_nd(c, A, r, s, n, delta);
    double pl[4] = {delta / tt, n[0], n[1], n[2]};
    if (st->tr && st->tr->n < st->tr->cap) {
        int k = st->tr->n++;
        st->tr->slots[k] = slot;
        memcpy(st->tr->planes + 4 * k, pl, sizeof pl);
        st->tr->energies[k] = E;
    }
    ++st->evaluated;
    if (st->best_slot < 0 || E > st->best_E) {
        if (st->best_slot >= 0) st->second_E = st->best_E;
        st->best_E = E;
        st->best_slot = slot;
        memcpy(st->best_plane, pl, sizeof pl);
    } else if (E > st->second_E) {
        st->second_E = E;
    }
}

/* candidate from the stored plane of cell k in the same view: the same 3D plane */
static void consider_cell(const slfo_ctx *c, const double *A, int r, int s, int k, int slot, argmax_t *st)
{
    const double *pk = A + 4 * gid(c, r, k);
    consider(c, A, r, s, pk + 1, plane_delta(c, r, k, pk), slot, st);
}

/* One refinement step of (r, s), Sec. III-C: propagation over the kernel
 * (current plane, the 8 ring neighbours, then far cells at distances
 * step, 2 step, ... <= R_I along the 8 ring directions), then 8 triangle
 * normals at the winner's centroid depth.  Slot numbers: 0 current, 1+j
 * ring, 9 + 8 (m/step - 1) + j far, 1000 + j normals. */
static int refine_one(const slfo_ctx *c, const double *A, int iter, int r, int s, double plane[4], double *energy,
                      int32_t *choice, double *margin, trace_t *tr, int pivot_slot)
{
    if (r < 0 || r >= c->V || s < 0 || s >= c->sp_off[r + 1] - c->sp_off[r] || iter < 1) return -1;
    int64_t g = gid(c, r, s);
    if (c->area[g] == 0) {
        plane[0] = plane[1] = plane[2] = plane[3] = 0.0;
        *energy = 0.0;
        *choice = -1;
        *margin = 0.0;
        return 0;
    }
    argmax_t st;
    st.best_E = -INFINITY;
    st.second_E = -INFINITY;
    st.best_slot = -1;
    st.evaluated = 0;
    st.tr = tr;
    memcpy(st.best_plane, A + 4 * g, sizeof st.best_plane);

    consider_cell(c, A, r, s, s, 0, &st);
    for (int j = 0; j < 8; ++j) {
        int k = cell_at(c, r, s, RING_DX[j], RING_DY[j]);
        if (k >= 0) consider_cell(c, A, r, s, k, 1 + j, &st);
    }
    int step = c->p.kernel_step;
    int RI = slfo_kernel_radius(c, r, iter);
    for (int m = step; m <= RI; m += step)
        for (int j = 0; j < 8; ++j) {
            int k = cell_at(c, r, s, m * RING_DX[j], m * RING_DY[j]);
            if (k >= 0) consider_cell(c, A, r, s, k, 9 + 8 * (m / step - 1) + j, &st);
        }

    /* Test hook: resolve the propagation stage toward `pivot_slot` (one of the
     * evaluated propagation slots), as a tie-break at a near-tie would. */
    if (pivot_slot >= 0 && tr) {
        int found = -1;
        for (int k = 0; k < tr->n; ++k)
            if (tr->slots[k] == pivot_slot) found = k;
        if (found < 0) return -2;
        st.best_slot = pivot_slot;
        st.best_E = tr->energies[found];
        memcpy(st.best_plane, tr->planes + 4 * found, sizeof st.best_plane);
        st.second_E = -INFINITY;
        st.evaluated = 1;
    }

    /* triangle normals through the 3D centroids of s (at the winner's depth)
     * and of two adjacent ring neighbours (at their depths in A) */
    if (st.best_slot >= 0) {
        const double *cs = c->cen + 2 * g;
        double rs[3], Xs[3];
        backproject(c, r, cs[0], cs[1], rs);
        double db = st.best_plane[0];
        for (int a = 0; a < 3; ++a) Xs[a] = db * rs[a];
        for (int j = 0; j < 8; ++j) {
            int ka = cell_at(c, r, s, RING_DX[j], RING_DY[j]);
            int kb = cell_at(c, r, s, RING_DX[(j + 1) % 8], RING_DY[(j + 1) % 8]);
            if (ka < 0 || kb < 0) continue;
            int64_t ga = gid(c, r, ka), gb = gid(c, r, kb);
            double ra[3], rb[3], ea[3], eb[3], nn[3];
            backproject(c, r, c->cen[2 * ga], c->cen[2 * ga + 1], ra);
            backproject(c, r, c->cen[2 * gb], c->cen[2 * gb + 1], rb);
            for (int a = 0; a < 3; ++a) {
                ea[a] = A[4 * ga] * ra[a] - Xs[a];
                eb[a] = A[4 * gb] * rb[a] - Xs[a];
            }
            nn[0] = ea[1] * eb[2] - ea[2] * eb[1];
            nn[1] = ea[2] * eb[0] - ea[0] * eb[2];
            nn[2] = ea[0] * eb[1] - ea[1] * eb[0];
            double len = sqrt(dot3(nn, nn));
            if (!(len > 1e-12 * sqrt(dot3(ea, ea)) * sqrt(dot3(eb, eb)))) continue;
            for (int a = 0; a < 3; ++a) nn[a] /= len;
            if (dot3(nn, rs) < 0.0)
                for (int a = 0; a < 3; ++a) nn[a] = -nn[a];
            consider(c, A, r, s, nn, dot3(nn, Xs), 1000 + j, &st);
        }
    }
    if (st.best_slot < 0) { /* invalid current plane and no valid candidate: keep A */
        memcpy(plane, A + 4 * g, 4 * sizeof(double));
        *energy = -INFINITY;
        *choice = -1;
        *margin = 0.0;
        return 0;
    }
    memcpy(plane, st.best_plane, sizeof st.best_plane);
    *energy = st.best_E;
    *choice = st.best_slot;
    *margin = st.evaluated > 1 ? st.best_E - st.second_E : INFINITY;
    return 0;
}

int slfo_refine_sp(const slfo_ctx *c, const double *A, int iter, int r, int s, double plane[4], double *energy,
                   int32_t *choice, double *margin)
{
    return refine_one(c, A, iter, r, s, plane, energy, choice, margin, NULL, -1);
}

int slfo_refine_trace(const slfo_ctx *c, const double *A, int iter, int r, int s, int32_t *slots, double *planes,
                      double *energies, int cap)
{
    trace_t tr = {slots, planes, energies, cap, 0};
    double pl[4], e, m;
    int32_t ch;
    int rc = refine_one(c, A, iter, r, s, pl, &e, &ch, &m, &tr, -1);
    return rc < 0 ? rc : tr.n;
}

int slfo_refine_pivot(const slfo_ctx *c, const double *A, int iter, int r, int s, int pivot_slot, double plane[4],
                      double *energy, int32_t *choice, int32_t *slots, double *planes, double *energies, int cap)
{
    trace_t tr = {slots, planes, energies, cap, 0};
    double m;
    int rc = refine_one(c, A, iter, r, s, plane, energy, choice, &m, &tr, pivot_slot);
    return rc < 0 ? rc : tr.n;
}

int slfo_refine_all(const slfo_ctx *c, const double *A, int iter, double *B, double *energy, int32_t *choice,
                    double *margin)
{
    int64_t S = c->S;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 2) reduction(| : bad)
    for (int64_t g = 0; g < S; ++g) {
        int v = 0;
        while (g >= c->sp_off[v + 1]) ++v;
        bad |= refine_one(c, A, iter, v, (int)(g - c->sp_off[v]), B + 4 * g, energy + g, choice + g, margin + g,
                          NULL, -1) != 0;
    }
    return bad ? -1 : 0;
}

/* --------------------------------------------------------- depth render */

/* D(p) = delta_s / (n_s . K^-1 p~) for s = label(p); 0 if not positive */
int slfo_render_depth(const slfo_ctx *c, const double *planes, int v, double *out)
{
    if (v < 0 || v >= c->V) return -1;
    int W = W_of(c, v), H = H_of(c, v);
    const int32_t *lab = lab_of(c, v);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int s = lab[(int64_t)y * W + x];
            const double *pl = planes + 4 * gid(c, v, s);
            double delta = plane_delta(c, v, s, pl);
            double ray[3];
            backproject(c, v, x, y, ray);
            double den = dot3(pl + 1, ray);
            double D = den > 0.0 ? delta / den : 0.0;
            out[(int64_t)y * W + x] = (D > 0.0 && isfinite(D)) ? D : 0.0;
        }
    return 0;
}
