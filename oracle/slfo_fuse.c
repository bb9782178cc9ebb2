/*
 * slfo_fuse — plain CPU oracle of the stability-based depth fusion that
 * follows the refinement (Chuchvara, Barsi, Gotchev, Sec. III-D; the two
 * passes per view of Sec. III-E).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Independent of
 * the HIP library (no shared code, headers or tables).
 *
 * What is computed, for one reference view r:
 *  1. Projection.  Every pixel q of every other view i with a depth D > 0 is
 *     lifted to its 3D point, moved into camera r and projected; the nearest
 *     pixel p of view r receives the point's depth in camera r as a
 *     candidate of view i.  Of several points of view i landing on p, the
 *     closest is kept (a depth test).  View r's own depth at p is its own
 *     candidate.
 *  2. Stability.  Each non-zero candidate c_j of p gains one for every other
 *     candidate of p that agrees with it, |c_k - c_j| <= tau c_j, and loses
 *     one for every other candidate that does not.  The fused depth is the
 *     smallest candidate whose stability is >= 0 (ties between equal depths:
 *     the smaller view index), 0 if none.
 *
 * Precision (the paper's depth maps are FP32 textures): depth maps and
 * candidates are FP32 values; the projection runs in FP64 and its result is
 * rounded to FP32; the agreement test is taken in FP32.  The projection
 * follows one fixed sequence of operations (stated below); the library must
 * build with -ffp-contract=off.
 */
#include "slfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Camera-r pixel and depth of pixel (u, v) of view i at depth D.  K = [[a b c]
 * [d e f] [0 0 1]]: the ray is (x, y, 1) with (x, y) the solution of
 * [[a b] [d e]] (x, y) = (u - c, v - f) by Cramer's rule; the point in camera
 * i is D (x, y, 1), in world coordinates R_i^T (X_i - t_i), in camera r
 * R_r X_w + t_r.  Returns 1 and the nearest pixel (round half up) and depth if
 * the point lies in front of camera r and inside its image, else 0. */
static int project_point(const int32_t *wh, const double *K, const double *R, const double *t, int i, int r,
                         double u, double v, double D, int *pu, int *pv, double *z)
{
    const double *Ki = K + 9 * i, *Ri = R + 9 * i, *ti = t + 3 * i;
    const double *Kr = K + 9 * r, *Rr = R + 9 * r, *tr = t + 3 * r;
    double du = u - Ki[2], dv = v - Ki[5];
    double det = Ki[0] * Ki[4] - Ki[1] * Ki[3];
    double x = (Ki[4] * du - Ki[1] * dv) / det;
    double y = (Ki[0] * dv - Ki[3] * du) / det;
    double Y[3] = {D * x - ti[0], D * y - ti[1], D - ti[2]};
    double Xw[3], Xr[3];
    for (int j = 0; j < 3; j++)
        Xw[j] = Ri[0 + j] * Y[0] + Ri[3 + j] * Y[1] + Ri[6 + j] * Y[2];
    for (int j = 0; j < 3; j++)
        Xr[j] = Rr[3 * j + 0] * Xw[0] + Rr[3 * j + 1] * Xw[1] + Rr[3 * j + 2] * Xw[2] + tr[j];
    if (!(Xr[2] > 0.0))
        return 0;
    double px = (Kr[0] * Xr[0] + Kr[1] * Xr[1] + Kr[2] * Xr[2]) / Xr[2];
    double py = (Kr[3] * Xr[0] + Kr[4] * Xr[1] + Kr[5] * Xr[2]) / Xr[2];
    double fu = floor(px + 0.5), fv = floor(py + 0.5);
    if (!(fu >= 0.0 && fu <= (double)(wh[2 * r] - 1) && fv >= 0.0 && fv <= (double)(wh[2 * r + 1] - 1)))
        return 0;
    *pu = (int)fu;
    *pv = (int)fv;
    *z = Xr[2];
    return 1;
}

static int64_t view_off(const int32_t *wh, int v)
{
    int64_t o = 0;
    for (int k = 0; k < v; k++)
        o += (int64_t)wh[2 * k] * wh[2 * k + 1];
    return o;
}

int slfo_fuse_project(int n_views, const int32_t *wh, const double *K, const double *R, const double *t,
                      const float *depth, int ref, int src, float *cand)
{
    if (n_views < 1 || ref < 0 || ref >= n_views || src < 0 || src >= n_views || src == ref)
        return -1;
    int Wr = wh[2 * ref], Hr = wh[2 * ref + 1], Ws = wh[2 * src], Hs = wh[2 * src + 1];
    const float *Ds = depth + view_off(wh, src);
    for (int64_t k = 0; k < (int64_t)Wr * Hr; k++)
        cand[k] = 0.0f;
    for (int v = 0; v < Hs; v++)
        for (int u = 0; u < Ws; u++) {
            float D = Ds[(int64_t)v * Ws + u];
            if (!(D > 0.0f) || isinf(D))
                continue;
            int pu, pv;
            double z;
            if (!project_point(wh, K, R, t, src, ref, (double)u, (double)v, (double)D, &pu, &pv, &z))
                continue;
            float zf = (float)z;
            if (!(zf > 0.0f) || isinf(zf))
                continue;
            float *slot = &cand[(int64_t)pv * Wr + pu];
            if (*slot == 0.0f || zf < *slot)
                *slot = zf;
        }
    return 0;
}

int slfo_fuse_vote(int n, const float *c, float tau, int32_t *stability)
{
    int best = -1;
    for (int j = 0; j < n; j++) {
        int32_t s = 0;
        if (!(c[j] > 0.0f)) {
            if (stability)
                stability[j] = 0;
            continue;
        }
        float lim = tau * c[j];
        for (int k = 0; k < n; k++) {
            if (k == j || !(c[k] > 0.0f))
                continue;
            float d = c[k] - c[j];
            if (d < 0.0f)
                d = -d;
            s += (d <= lim) ? 1 : -1;
        }
        if (stability)
            stability[j] = s;
        if (s >= 0 && (best < 0 || c[j] < c[best]))
            best = j;
    }
    return best;
}

int slfo_fuse_view(int n_views, const int32_t *wh, const double *K, const double *R, const double *t,
                   const float *depth, int ref, float tau, float *fused, int32_t *winner, int32_t *stability,
                   int32_t *n_cand)
{
    if (n_views < 1 || n_views > 64 || ref < 0 || ref >= n_views || !(tau >= 0.0f))
        return -1;
    int64_t P = (int64_t)wh[2 * ref] * wh[2 * ref + 1];
    float *layers = (float *)malloc(sizeof(float) * (size_t)(P * n_views));
    if (!layers)
        return -3;
    const float *Dr = depth + view_off(wh, ref);
    int rc = 0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n_views; i++) {
        float *L = layers + (int64_t)i * P;
        if (i == ref) {
            for (int64_t k = 0; k < P; k++)
                L[k] = (Dr[k] > 0.0f && !isinf(Dr[k])) ? Dr[k] : 0.0f;
        } else if (slfo_fuse_project(n_views, wh, K, R, t, depth, ref, i, L)) {
            rc = -1;
        }
    }
    if (rc) {
        free(layers);
        return rc;
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < P; k++) {
        float c[64];
        int32_t s[64];
        int n = n_views;
        int m = 0;
        for (int i = 0; i < n; i++) {
            c[i] = layers[(int64_t)i * P + k];
            m += c[i] > 0.0f;
        }
        int b = slfo_fuse_vote(n, c, tau, s);
        fused[k] = b >= 0 ? c[b] : 0.0f;
        if (winner)
            winner[k] = b;
        if (stability)
            stability[k] = b >= 0 ? s[b] : 0;
        if (n_cand)
            n_cand[k] = m;
    }
    free(layers);
    return 0;
}
