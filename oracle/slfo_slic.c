/*
 * slfo_slic — plain CPU oracle of the grid-seeded SLIC segmentation the method
 * starts from (Chuchvara, Barsi, Gotchev, Sec. III-A: SLIC superpixels read as
 * an approximately regular grid of cells; the GPU SLIC of Sec. III-E).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Independent of
 * the HIP library (no shared code, headers or tables).
 *
 * SLIC (simple linear iterative clustering) as used here:
 *  - one cluster per cell (gx, gy) of a gw x gh grid over the W x H image,
 *    keeping the cell id k = gy gw + gx as its label; its centre starts at
 *    the cell centre ((gx + 0.5) W / gw - 0.5, (gy + 0.5) H / gh - 0.5) with
 *    the colour of the pixel nearest to it (round half up);
 *  - assignment: pixel (u, v) lies in cell (floor((u + 0.5) gw / W), floor((v
 *    + 0.5) gh / H)) and takes the label of the closest centre among the 3 x
 *    3 cells around it, distance D = |rgb - rgb_k|^2 + ((u - u_k)^2 + (v -
 *    v_k)^2) w with w = (2.55 m)^2 gw gh / (W H) (m the compactness, colours in
 *    0..255; the same D as colours in 0..100 with spatial weight m^2 / S^2);
 *    ties go to the first centre in the order dy = -1..1, dx = -1..1;
 *  - update: each centre becomes the mean position and colour of its pixels
 *    (a centre without pixels stays);
 *  - after the iterations, connectivity: for each label only its largest
 *    4-connected component keeps it (equal sizes: the component whose first
 *    pixel in raster order comes first); every other component takes the
 *    final label of the component holding the pixel left of its first pixel,
 *    or the pixel above it in the first column (both lie in another label:
 *    a same-label neighbour would belong to the component and come first).
 *    A component whose first pixel is the image's first pixel keeps its
 *    label.
 *
 * Precision.  The decisions are integer (labels); both sides take them in
 * FP32: sums of positions and colours are exact integers, a centre is
 * (float)sum / (float)count, and D is evaluated in the order written above
 * with FP32 operations (build with -ffp-contract=off).
 */
#include "slfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int cell_of(int p, int n, int g)
{
    /* floor((p + 0.5) g / n) = floor((2p + 1) g / (2n)) in integers */
    int c = (int)(((int64_t)(2 * p + 1) * g) / (2 * (int64_t)n));
    return c < g ? c : g - 1;
}

float slfo_slic_weight(int W, int H, int gw, int gh, double compactness)
{
    double m = 2.55 * compactness;
    return (float)(m * m * (double)gw * (double)gh / ((double)W * (double)H));
}

/* one assignment pass: labels from centres cen[k] = (u, v, r, g, b) (FP32) */
static void assign(int W, int H, const uint8_t *rgb, int gw, int gh, const float *cen, float wsp, int32_t *labels)
{
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        int cy = cell_of(v, H, gh);
        for (int u = 0; u < W; ++u) {
            int cx = cell_of(u, W, gw);
            const uint8_t *p = rgb + 3 * ((int64_t)v * W + u);
            float best = INFINITY;
            int bk = cy * gw + cx;
            for (int dy = -1; dy <= 1; ++dy) {
                int gy = cy + dy;
                if (gy < 0 || gy >= gh) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    int gx = cx + dx;
                    if (gx < 0 || gx >= gw) continue;
                    int k = gy * gw + gx;
                    const float *c = cen + 5 * k;
                    float du = (float)u - c[0], dv = (float)v - c[1];
                    float d0 = (float)p[0] - c[2], d1 = (float)p[1] - c[3], d2 = (float)p[2] - c[4];
                    float dc = d0 * d0 + d1 * d1 + d2 * d2;
                    float ds = du * du + dv * dv;
                    float D = dc + ds * wsp;
                    if (D < best) {
                        best = D;
                        bk = k;
                    }
                }
            }
            labels[(int64_t)v * W + u] = bk;
        }
    }
}

int slfo_slic_centres_init(int W, int H, const uint8_t *rgb, int gw, int gh, float *cen)
{
    if (W < 1 || H < 1 || gw < 1 || gh < 1 || gw > W || gh > H) return -1;
    for (int k = 0; k < gw * gh; ++k) {
        int gx = k % gw, gy = k / gw;
        double u = (gx + 0.5) * (double)W / gw - 0.5, v = (gy + 0.5) * (double)H / gh - 0.5;
        int iu = (int)floor(u + 0.5), iv = (int)floor(v + 0.5);
        if (iu > W - 1) iu = W - 1;
        if (iv > H - 1) iv = H - 1;
        const uint8_t *p = rgb + 3 * ((int64_t)iv * W + iu);
        cen[5 * k + 0] = (float)u;
        cen[5 * k + 1] = (float)v;
        for (int c = 0; c < 3; ++c) cen[5 * k + 2 + c] = (float)p[c];
    }
    return 0;
}

int slfo_slic_assign(int W, int H, const uint8_t *rgb, int gw, int gh, const float *cen, double compactness,
                     int32_t *labels)
{
    if (W < 1 || H < 1 || gw < 1 || gh < 1 || gw > W || gh > H) return -1;
    assign(W, H, rgb, gw, gh, cen, slfo_slic_weight(W, H, gw, gh, compactness), labels);
    return 0;
}

int slfo_slic_update(int W, int H, const uint8_t *rgb, int gw, int gh, const int32_t *labels, float *cen)
{
    int K = gw * gh;
    int64_t *acc = (int64_t *)calloc((size_t)K * 6, sizeof(int64_t));
    if (!acc) return -3;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int64_t i = (int64_t)v * W + u;
            int k = labels[i];
            if (k < 0 || k >= K) {
                free(acc);
                return -2;
            }
            int64_t *a = acc + 6 * k;
            a[0] += u;
            a[1] += v;
            a[2] += rgb[3 * i];
            a[3] += rgb[3 * i + 1];
            a[4] += rgb[3 * i + 2];
            a[5] += 1;
        }
    for (int k = 0; k < K; ++k) {
        int64_t n = acc[6 * k + 5];
        if (n > 0)
            for (int c = 0; c < 5; ++c) cen[5 * k + c] = (float)acc[6 * k + c] / (float)n;
    }
    free(acc);
    return 0;
}

int slfo_slic_connectivity(int W, int H, int gw, int gh, int32_t *labels)
{
    int64_t N = (int64_t)W * H;
    int K = gw * gh;
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *csize = (int32_t *)malloc(sizeof(int32_t) * N);  /* per component id = its first pixel */
    int32_t *keep = (int32_t *)malloc(sizeof(int32_t) * K);
    int32_t *final = (int32_t *)malloc(sizeof(int32_t) * N);
    if (!comp || !queue || !csize || !keep || !final) {
        free(comp); free(queue); free(csize); free(keep); free(final);
        return -3;
    }
    static const int du4[4] = {1, -1, 0, 0}, dv4[4] = {0, 0, 1, -1};
    for (int64_t i = 0; i < N; ++i) comp[i] = -1;
    /* components by breadth-first search, named by their first pixel in raster order */
    for (int64_t s = 0; s < N; ++s) {
        if (comp[s] >= 0) continue;
        int lab = labels[s];
        int64_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        comp[s] = (int32_t)s;
        while (head < tail) {
            int32_t q = queue[head++];
            int qu = q % W, qv = q / W;
            for (int d = 0; d < 4; ++d) {
                int nu = qu + du4[d], nv = qv + dv4[d];
                if (nu < 0 || nu >= W || nv < 0 || nv >= H) continue;
                int64_t ni = (int64_t)nv * W + nu;
                if (comp[ni] < 0 && labels[ni] == lab) {
                    comp[ni] = (int32_t)s;
                    queue[tail++] = (int32_t)ni;
                }
            }
        }
        csize[s] = (int32_t)tail;
    }
    /* the largest component of each label (equal sizes: the earlier first pixel) */
    for (int k = 0; k < K; ++k) keep[k] = -1;
    for (int64_t s = 0; s < N; ++s) {
        if (comp[s] != s) continue;
        int k = labels[s];
        if (keep[k] < 0 || csize[s] > csize[keep[k]]) keep[k] = (int32_t)s;
    }
    /* final labels in raster order of the components' first pixels: the pixel
     * left of (or above) a first pixel lies in a component with an earlier
     * first pixel, whose final label is already known */
    for (int64_t s = 0; s < N; ++s) {
        if (comp[s] != s) continue;
        int k = labels[s];
        if (keep[k] == s || s == 0) {
            final[s] = k;
            continue;
        }
        int u = (int)(s % W);
        int64_t nb = u > 0 ? s - 1 : s - W;
        final[s] = final[comp[nb]];
    }
    for (int64_t i = 0; i < N; ++i) labels[i] = final[comp[i]];
    free(comp); free(queue); free(csize); free(keep); free(final);
    return 0;
}

int slfo_slic(int W, int H, const uint8_t *rgb, int gw, int gh, int iterations, double compactness,
              int connectivity, int32_t *labels)
{
    if (W < 1 || H < 1 || gw < 1 || gh < 1 || gw > W || gh > H || iterations < 1 || !(compactness >= 0.0))
        return -1;
    float *cen = (float *)malloc(sizeof(float) * 5 * (size_t)gw * gh);
    if (!cen) return -3;
    slfo_slic_centres_init(W, H, rgb, gw, gh, cen);
    float wsp = slfo_slic_weight(W, H, gw, gh, compactness);
    for (int it = 0; it < iterations; ++it) {
        assign(W, H, rgb, gw, gh, cen, wsp, labels);
        if (it + 1 < iterations) slfo_slic_update(W, H, rgb, gw, gh, labels, cen);
    }
    free(cen);
    return connectivity ? slfo_slic_connectivity(W, H, gw, gh, labels) : 0;
}
