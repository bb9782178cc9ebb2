/*
 * Seeded synthetic light-field inputs: a ray caster for scenes of textured
 * rectangles and a grid-seeded SLIC over-segmentation whose labels keep the
 * seed-grid cell ids.
 *
 * This file makes INPUTS only.  It contains none of the depth method's
 * arithmetic (no homographies, no matching costs, no energies), and both the
 * FP64 oracle and the HIP library consume what it produces.
 *
 * Texture noise uses the MurmurHash3 64-bit finaliser (fmix64, Appleby 2011)
 * on lattice coordinates, so textures of unbounded planes need no storage.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/* Integer lattice hash -> uniform integer in [0, 255]. */
static int lattice_u8(uint64_t seed, int64_t ix, int64_t iy, int ch)
{
    uint64_t h = fmix64(seed ^ fmix64((uint64_t)ix * 0x9E3779B97F4A7C15ULL ^
                                      fmix64((uint64_t)iy + 0x632BE59BD9B4E019ULL) ^
                                      ((uint64_t)ch << 56)));
    return (int)(h >> 56);
}

static double smooth(double f) { return f * f * (3.0 - 2.0 * f); }

/* Value noise in [0,255]: smoothstep-weighted blend of four lattice values. */
static double value_noise(uint64_t seed, double a, double b, double cell, int ch)
{
    double x = a / cell, y = b / cell;
    double fx0 = floor(x), fy0 = floor(y);
    int64_t ix = (int64_t)fx0, iy = (int64_t)fy0;
    double sx = smooth(x - fx0), sy = smooth(y - fy0);
    double v00 = lattice_u8(seed, ix, iy, ch), v10 = lattice_u8(seed, ix + 1, iy, ch);
    double v01 = lattice_u8(seed, ix, iy + 1, ch), v11 = lattice_u8(seed, ix + 1, iy + 1, ch);
    double top = v00 + sx * (v10 - v00);
    double bot = v01 + sx * (v11 - v01);
    return top + sy * (bot - top);
}

/*
 * One scene rectangle, 20 doubles:
 *  [0..2] centre P0, [3..5] in-plane axis e1, [6..8] in-plane axis e2,
 *  [9..11] unit normal n = e1 x e2, [12] half extent along e1, [13] along e2
 *  (<= 0 means unbounded), [14] texture kind (0 = two-octave value noise,
 *  1 = constant colour + integer texel noise in [-2,2]), [15] coarse cell /
 *  texel pitch (world units), [16] fine cell (world units), [17..19] constant
 *  colour (kind 1).  tex_seed[j] seeds the lattice of rectangle j.
 */
#define RECT_STRIDE 20

static void shade(const double *pl, uint64_t seed, double a, double b, uint8_t *rgb)
{
    int kind = (int)pl[14];
    for (int c = 0; c < 3; ++c) {
        double v;
        if (kind == 0) {
            v = 0.55 * value_noise(seed, a, b, pl[15], c) + 0.45 * value_noise(seed ^ 0xABCDEFULL, a, b, pl[16], c);
        } else {
            int64_t ix = (int64_t)floor(a / pl[15]), iy = (int64_t)floor(b / pl[15]);
            int noise = lattice_u8(seed, ix, iy, c) % 5 - 2;
            v = pl[17 + c] + noise;
        }
        long q = lround(v);
        if (q < 0) q = 0;
        if (q > 255) q = 255;
        rgb[c] = (uint8_t)q;
    }
}

/*
 * Ray-cast one pinhole view.  Camera convention: X_cam = R X_world + t and
 * pixel ~ K X_cam with pixel centres at integer (u, v).  Outputs RGB8, the
 * camera-z depth of the nearest hit (0 where nothing is hit) and the index of
 * the rectangle hit (-1 where nothing is hit).
 */
void synth_raycast(int W, int H, const double *K, const double *R, const double *t,
                   int n_rect, const double *rects, const uint64_t *tex_seed,
                   uint8_t *rgb, double *depth, int32_t *plane_id)
{
    double fx = K[0], sk = K[1], cx = K[2], fy = K[4], cy = K[5];
    double C[3];
    for (int k = 0; k < 3; ++k)
        C[k] = -(R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1] + R[2 * 3 + k] * t[2]);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            /* camera-frame ray with unit z, then to world */
            double yc = (v - cy) / fy;
            double xc = (u - cx - sk * yc) / fx;
            double dc[3] = {xc, yc, 1.0};
            double dw[3];
            for (int k = 0; k < 3; ++k)
                dw[k] = R[0 * 3 + k] * dc[0] + R[1 * 3 + k] * dc[1] + R[2 * 3 + k] * dc[2];
            double best = INFINITY;
            int best_j = -1;
            double best_a = 0, best_b = 0;
            for (int j = 0; j < n_rect; ++j) {
                const double *pl = rects + (size_t)j * RECT_STRIDE;
                double den = pl[9] * dw[0] + pl[10] * dw[1] + pl[11] * dw[2];
                if (fabs(den) < 1e-12) continue;
                double num = pl[9] * (pl[0] - C[0]) + pl[10] * (pl[1] - C[1]) + pl[11] * (pl[2] - C[2]);
                double th = num / den;
                if (!(th > 1e-9) || th >= best) continue;
                double X[3] = {C[0] + th * dw[0] - pl[0], C[1] + th * dw[1] - pl[1], C[2] + th * dw[2] - pl[2]};
                double a = X[0] * pl[3] + X[1] * pl[4] + X[2] * pl[5];
                double b = X[0] * pl[6] + X[1] * pl[7] + X[2] * pl[8];
                if (pl[12] > 0 && fabs(a) > pl[12]) continue;
                if (pl[13] > 0 && fabs(b) > pl[13]) continue;
                best = th;
                best_j = j;
                best_a = a;
                best_b = b;
            }
            size_t idx = (size_t)v * W + u;
            if (best_j >= 0) {
                shade(rects + (size_t)best_j * RECT_STRIDE, tex_seed[best_j], best_a, best_b, rgb + 3 * idx);
                depth[idx] = best; /* dc has unit z, so the ray parameter is camera z */
                plane_id[idx] = best_j;
            } else {
                rgb[3 * idx] = rgb[3 * idx + 1] = rgb[3 * idx + 2] = 0;
                depth[idx] = 0.0;
                plane_id[idx] = -1;
            }
        }
    }
}

/*
 * Grid-seeded SLIC (Achanta et al. 2012) on RGB.  Cluster k starts at the
 * centre of grid cell (k mod gw, k div gw); each pixel compares the centres of
 * the 3x3 cells around its own cell; labels keep the cell ids.  Distance:
 * dc^2 + (ds / S)^2 * m^2 with colour in [0,100]-scaled RGB units.  After the
 * iterations, each label keeps its largest 4-connected component and every
 * other fragment is merged into the label of an adjacent final component.
 * Returns the number of labels left without pixels.
 */
int synth_slic(int W, int H, const uint8_t *rgb, int gw, int gh, int iters, double compactness,
               int32_t *labels)
{
    int K = gw * gh;
    double sx = (double)W / gw, sy = (double)H / gh;
    double S = sqrt((double)W * H / K);
    double *cen = (double *)malloc(sizeof(double) * 5 * K);
    double *acc = (double *)malloc(sizeof(double) * 6 * K);
    const double cs = 100.0 / 255.0;
    const double wspace = compactness * compactness / (S * S);
    for (int k = 0; k < K; ++k) {
        int gx = k % gw, gy = k / gw;
        double u = (gx + 0.5) * sx - 0.5, v = (gy + 0.5) * sy - 0.5;
        int iu = (int)lround(u), iv = (int)lround(v);
        if (iu < 0) iu = 0;
        if (iu >= W) iu = W - 1;
        if (iv < 0) iv = 0;
        if (iv >= H) iv = H - 1;
        const uint8_t *p = rgb + 3 * ((size_t)iv * W + iu);
        cen[5 * k + 0] = u;
        cen[5 * k + 1] = v;
        for (int c = 0; c < 3; ++c) cen[5 * k + 2 + c] = p[c] * cs;
    }
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int v = 0; v < H; ++v) {
            int cy = (int)floor((v + 0.5) / sy);
            if (cy >= gh) cy = gh - 1;
            for (int u = 0; u < W; ++u) {
                int cx = (int)floor((u + 0.5) / sx);
                if (cx >= gw) cx = gw - 1;
                const uint8_t *p = rgb + 3 * ((size_t)v * W + u);
                double best = INFINITY;
                int bk = cy * gw + cx;
                for (int dy = -1; dy <= 1; ++dy) {
                    int gy = cy + dy;
                    if (gy < 0 || gy >= gh) continue;
                    for (int dx = -1; dx <= 1; ++dx) {
                        int gx = cx + dx;
                        if (gx < 0 || gx >= gw) continue;
                        int k = gy * gw + gx;
                        const double *c = cen + 5 * k;
                        double du = u - c[0], dv = v - c[1];
                        double d0 = p[0] * cs - c[2], d1 = p[1] * cs - c[3], d2 = p[2] * cs - c[4];
                        double D = d0 * d0 + d1 * d1 + d2 * d2 + (du * du + dv * dv) * wspace;
                        if (D < best) {
                            best = D;
                            bk = k;
                        }
                    }
                }
                labels[(size_t)v * W + u] = bk;
            }
        }
        memset(acc, 0, sizeof(double) * 6 * K);
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                size_t i = (size_t)v * W + u;
                double *a = acc + 6 * labels[i];
                a[0] += u;
                a[1] += v;
                a[2] += rgb[3 * i] * cs;
                a[3] += rgb[3 * i + 1] * cs;
                a[4] += rgb[3 * i + 2] * cs;
                a[5] += 1.0;
            }
        for (int k = 0; k < K; ++k) {
            double n = acc[6 * k + 5];
            if (n > 0)
                for (int c = 0; c < 5; ++c) cen[5 * k + c] = acc[6 * k + c] / n;
        }
    }
    free(cen);
    free(acc);

    /* connectivity: 4-connected components */
    size_t N = (size_t)W * H;
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * N);
    for (size_t i = 0; i < N; ++i) comp[i] = -1;
    int ncomp = 0, cap = 1024;
    int32_t *csize = (int32_t *)malloc(sizeof(int32_t) * cap);
    int32_t *clabel = (int32_t *)malloc(sizeof(int32_t) * cap);
    int32_t *cfirst = (int32_t *)malloc(sizeof(int32_t) * cap);
    static const int du4[4] = {1, -1, 0, 0}, dv4[4] = {0, 0, 1, -1};
    for (size_t s = 0; s < N; ++s) {
        if (comp[s] >= 0) continue;
        if (ncomp == cap) {
            cap *= 2;
            csize = (int32_t *)realloc(csize, sizeof(int32_t) * cap);
            clabel = (int32_t *)realloc(clabel, sizeof(int32_t) * cap);
            cfirst = (int32_t *)realloc(cfirst, sizeof(int32_t) * cap);
        }
        int lab = labels[s];
        size_t head = 0, tail = 0;
        queue[tail++] = (int32_t)s;
        comp[s] = ncomp;
        while (head < tail) {
            int32_t q = queue[head++];
            int qu = q % W, qv = q / W;
            for (int d = 0; d < 4; ++d) {
                int nu = qu + du4[d], nv = qv + dv4[d];
                if (nu < 0 || nu >= W || nv < 0 || nv >= H) continue;
                size_t ni = (size_t)nv * W + nu;
                if (comp[ni] < 0 && labels[ni] == lab) {
                    comp[ni] = ncomp;
                    queue[tail++] = (int32_t)ni;
                }
            }
        }
        csize[ncomp] = (int32_t)tail;
        clabel[ncomp] = lab;
        cfirst[ncomp] = (int32_t)s;
        ++ncomp;
    }
    int32_t *main_comp = (int32_t *)malloc(sizeof(int32_t) * K);
    for (int k = 0; k < K; ++k) main_comp[k] = -1;
    for (int c = 0; c < ncomp; ++c) {
        int k = clabel[c];
        if (main_comp[k] < 0 || csize[c] > csize[main_comp[k]]) main_comp[k] = c;
    }
    /* final[c]: label a component ends with, or -1 while unresolved */
    int32_t *final_lab = (int32_t *)malloc(sizeof(int32_t) * ncomp);
    int unresolved = 0;
    for (int c = 0; c < ncomp; ++c) {
        final_lab[c] = (main_comp[clabel[c]] == c) ? clabel[c] : -1;
        if (final_lab[c] < 0) ++unresolved;
    }
    while (unresolved > 0) {
        int progress = 0;
        for (int c = 0; c < ncomp; ++c) {
            if (final_lab[c] >= 0) continue;
            /* flood the fragment again and take the first resolved neighbour */
            size_t head = 0, tail = 0;
            int32_t s = cfirst[c];
            queue[tail++] = s;
            int found = -1;
            /* visited marker: temporarily negate comp ids to -(c+2) */
            comp[s] = -(c + 2);
            while (head < tail) {
                int32_t q = queue[head++];
                int qu = q % W, qv = q / W;
                for (int d = 0; d < 4; ++d) {
                    int nu = qu + du4[d], nv = qv + dv4[d];
                    if (nu < 0 || nu >= W || nv < 0 || nv >= H) continue;
                    size_t ni = (size_t)nv * W + nu;
                    int cn = comp[ni];
                    if (cn == c) {
                        comp[ni] = -(c + 2);
                        queue[tail++] = (int32_t)ni;
                    } else if (cn >= 0 && final_lab[cn] >= 0 && found < 0) {
                        found = final_lab[cn];
                    }
                }
            }
            for (size_t h = 0; h < tail; ++h) comp[queue[h]] = c;
            if (found >= 0) {
                final_lab[c] = found;
                --unresolved;
                progress = 1;
            }
        }
        if (!progress) break; /* cannot happen on a connected image */
    }
    for (size_t i = 0; i < N; ++i) {
        int f = final_lab[comp[i]];
        labels[i] = f >= 0 ? f : clabel[comp[i]];
    }
    int empty = 0;
    int32_t *cnt = (int32_t *)calloc(K, sizeof(int32_t));
    for (size_t i = 0; i < N; ++i) cnt[labels[i]]++;
    for (int k = 0; k < K; ++k) empty += cnt[k] == 0;
    free(cnt);
    free(final_lab);
    free(main_comp);
    free(csize);
    free(clabel);
    free(cfirst);
    free(comp);
    free(queue);
    return empty;
}
