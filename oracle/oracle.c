/*
 * CPU oracle for the StereoVAE hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, scalar loops that state each operation as its definition.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no source, header or helper with the GPU
 * library: it has its own declarations below and is built by gcc, not hipcc.
 *
 * Integer steps (downsample, census, Hamming cost, winner-take-all) are exact.
 * Network primitives (convolution, bilinear resize and their adjoints) work in
 * FP64 on NCHW arrays; the network is composed from them in oracle/vae.py.
 *
 * Pins: every function here is checked by the CPU tests against brute force,
 * closed forms, invariants or an independent library routine (torch CPU
 * float64), never against the GPU library.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Matching: the coarse disparity map of Sec. III-A, computed on the reduced */
/* ("small") image pair.                                                      */
/* ------------------------------------------------------------------------ */

/* Reduced-resolution image ("small image pairs", Sec. IV-C; quarter-size
 * inputs, Table I).  The paper does not state the filter; this is the f x f
 * block mean with round-half-up, partial edge blocks averaged over their
 * in-bounds pixels.  out[b][i][j] for i < ceil(H/f), j < ceil(W/f). */
void or_downsample(const uint8_t *img, int B, int H, int W, int pitch, int f, uint8_t *out)
{
    int h = (H + f - 1) / f, w = (W + f - 1) / f;
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j) {
                long S = 0, n = 0;
                for (int y = f * i; y < f * i + f && y < H; ++y)
                    for (int x = f * j; x < f * j + f && x < W; ++x) {
                        S += img[(size_t)b * H * pitch + (size_t)y * pitch + x];
                        ++n;
                    }
                out[((size_t)b * h + i) * w + j] = (uint8_t)((S + n / 2) / n);
            }
}

/* Census transform (named in Sec. I and Sec. III; robustness variants S1/S2 of
 * Sec. IV-C).  Window win_w wide and win_h tall, both odd; offsets enumerated
 * row by row (dy outer, dx inner) skipping the centre, bit k set when the
 * k-th neighbour is strictly darker than the centre.  Borders clamp to the
 * edge.  Bits at and above nbits = win_w*win_h - 1 are zero. */
void or_census(const uint8_t *img, int B, int h, int w, int win_w, int win_h, uint64_t *out)
{
    int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j) {
                const uint8_t *im = img + (size_t)b * h * w;
                int centre = im[(size_t)i * w + j];
                uint64_t code = 0;
                int k = 0;
                for (int dy = -ry; dy <= ry; ++dy)
                    for (int dx = -rx; dx <= rx; ++dx) {
                        if (dy == 0 && dx == 0)
                            continue;
                        int y = clampi(i + dy, 0, h - 1), x = clampi(j + dx, 0, w - 1);
                        if (im[(size_t)y * w + x] < centre)
                            code |= (uint64_t)1 << k;
                        ++k;
                    }
                out[((size_t)b * h + i) * w + j] = code;
            }
}

static int popcount64(uint64_t v)
{
    int c = 0;
    while (v) {
        c += (int)(v & 1u);
        v >>= 1;
    }
    return c;
}

/* Matching cost volume C(x, y, d) between reference pixel (x, y) of the left
 * view and target pixel (x - d, y) of the right view (the indexing of Eq. (1)
 * and Eq. (4)), here the Hamming distance of census codes.  A target column
 * outside the image costs nbits + 1.  cost[b][i][j][d], d < D. */
void or_cost_volume(const uint64_t *cl, const uint64_t *cr, int B, int h, int w, int D, int nbits,
                    int32_t *cost)
{
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j)
                for (int d = 0; d < D; ++d) {
                    size_t o = (((size_t)b * h + i) * w + j) * D + d;
                    if (j - d < 0)
                        cost[o] = nbits + 1;
                    else
                        cost[o] = popcount64(cl[((size_t)b * h + i) * w + j] ^
                                             cr[((size_t)b * h + i) * w + (j - d)]);
                }
}

/* Winner-take-all, Eq. (6): the disparity of least cost, the lowest one on ties. */
void or_wta(const int32_t *cost, int B, int h, int w, int D, uint8_t *disp)
{
    for (size_t p = 0; p < (size_t)B * h * w; ++p) {
        int best = 0;
        for (int d = 1; d < D; ++d)
            if (cost[p * D + d] < cost[p * D + best])
                best = d;
        disp[p] = (uint8_t)best;
    }
}

/* ------------------------------------------------------------------------ */
/* Semi-global matching and post-processing (Sec. III-A2, III-A3), the      */
/* Census + SGM member of the paper's family (S2 of Sec. IV-C).               */
/* ------------------------------------------------------------------------ */

/* Path cost along one direction r, Eq. (4):
 *   C_r(p, d) = C(p, d) + min(C_r(p - r, d), C_r(p - r, d - 1) + P1,
 *                             C_r(p - r, d + 1) + P1, min_i C_r(p - r, i) + P2)
 *               - min_k C_r(p - r, k),
 * with C_r(p, d) = C(p, d) at the first pixel of each path and the d - 1 /
 * d + 1 terms absent outside [0, D).  Directions: 0 = left to right (r is one
 * column back), 1 = right to left, 2 = top to bottom, 3 = bottom to top.
 * cost and out are [B][h][w][D]. */
void or_sgm_path(const int32_t *cost, int B, int h, int w, int D, int P1, int P2, int dir,
                 int32_t *out)
{
    const int dy = dir == 2 ? 1 : (dir == 3 ? -1 : 0);
    const int dx = dir == 0 ? 1 : (dir == 1 ? -1 : 0);
    for (int b = 0; b < B; ++b) {
        /* visit pixels in path order: the predecessor p - r is always done */
        for (int ii = 0; ii < h; ++ii)
            for (int jj = 0; jj < w; ++jj) {
                const int i = dy < 0 ? h - 1 - ii : ii;
                const int j = dx < 0 ? w - 1 - jj : jj;
                const int pi = i - dy, pj = j - dx;
                const size_t o = (((size_t)b * h + i) * w + j) * D;
                if (pi < 0 || pi >= h || pj < 0 || pj >= w) {
                    for (int d = 0; d < D; ++d) out[o + d] = cost[o + d];
                    continue;
                }
                const int32_t *prev = out + (((size_t)b * h + pi) * w + pj) * D;
                int32_t mprev = prev[0];
                for (int k = 1; k < D; ++k)
                    if (prev[k] < mprev) mprev = prev[k];
                for (int d = 0; d < D; ++d) {
                    int32_t m = prev[d];
                    if (d > 0 && prev[d - 1] + P1 < m) m = prev[d - 1] + P1;
                    if (d + 1 < D && prev[d + 1] + P1 < m) m = prev[d + 1] + P1;
                    if (mprev + P2 < m) m = mprev + P2;
                    out[o + d] = cost[o + d] + m - mprev;
                }
            }
    }
}

/* Aggregated cost, Eq. (5): C_SGM(p, d) = sum over the directions of C_r(p, d)
 * (paths: the four axis directions). */
void or_sgm(const int32_t *cost, int B, int h, int w, int D, int P1, int P2, int32_t *sum,
            int32_t *scratch)
{
    const size_t n = (size_t)B * h * w * D;
    for (size_t k = 0; k < n; ++k) sum[k] = 0;
    for (int dir = 0; dir < 4; ++dir) {
        or_sgm_path(cost, B, h, w, D, P1, P2, dir, scratch);
        for (size_t k = 0; k < n; ++k) sum[k] += scratch[k];
    }
}

/* Single matching phase, Eq. (7), as read here: the target column of (x, y) is
 * x - D(x, y), and no target column may be matched twice.  When two reference
 * pixels x < x' of a row share a target column, x' has the larger disparity
 * and hides x in the target view, so x is the occluded one: (x, y) is invalid
 * when some pixel (x + k, y), 0 < k < D, has the same target column.  An
 * invalid value is replaced by the nearest valid value of the same row (on
 * equal distances the smaller of the two); a row with no valid pixel is left
 * as it is. */
void or_smp(const uint8_t *disp, int B, int h, int w, int D, uint8_t *out)
{
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i) {
            const uint8_t *row = disp + ((size_t)b * h + i) * w;
            uint8_t *orow = out + ((size_t)b * h + i) * w;
            int any = 0;
            /* valid[] kept in the output's spare values: 1 = valid */
            static unsigned char valid[1 << 16];
            for (int x = 0; x < w; ++x) {
                int ok = 1;
                for (int k = 1; k < D && x + k < w; ++k)
                    if ((x + k) - row[x + k] == x - row[x]) ok = 0;
                valid[x] = (unsigned char)ok;
                any |= ok;
            }
            for (int x = 0; x < w; ++x) {
                if (valid[x] || !any) {
                    orow[x] = row[x];
                    continue;
                }
                int best = -1;
                for (int dist = 1; best < 0; ++dist) {
                    const int l = x - dist, r = x + dist;
                    const int lv = l >= 0 && valid[l], rv = r < w && valid[r];
                    if (lv && rv) best = row[l] < row[r] ? row[l] : row[r];
                    else if (lv) best = row[l];
                    else if (rv) best = row[r];
                }
                orow[x] = (uint8_t)best;
            }
        }
}

/* Zero-mean normalised cross-correlation cost, Eqs. (1)-(3), on the reduced
 * images, window win_w x win_h centred on each pixel, window pixels clamped to
 * the image edge, target pixel (x - d, y):
 *   C = 1 - sum dR dT / (sigma_R sigma_T),  dR = I_R - mean_W(I_R), ...
 * With n window pixels and exact integer sums SR, SRR, ST, STT, SRT,
 *   sum dR dT = (n SRT - SR ST) / n,  sigma_R^2 = (n SRR - SR^2) / n, ...
 * so C = 1 - N / sqrt(A B) with N = n SRT - SR ST, A = n SRR - SR^2,
 * B = n STT - ST^2 (exact integers, then FP64).  A flat window (A or B zero)
 * carries no correlation: C = 1.  A target column outside the image: C = 2.
 * The cost kept for the path aggregation is q = floor(32 C + 1/2) in 0..64
 * (FP64), out[b][i][j][d]. */
void or_zncc_cost(const uint8_t *ll, const uint8_t *lr, int B, int h, int w, int D, int win_w,
                  int win_h, int32_t *out)
{
    const int rx = (win_w - 1) / 2, ry = (win_h - 1) / 2;
    const long long n = (long long)win_w * win_h;
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j)
                for (int d = 0; d < D; ++d) {
                    double C;
                    if (j - d < 0) {
                        C = 2.0;
                    } else {
                        long long SR = 0, SRR = 0, ST = 0, STT = 0, SRT = 0;
                        for (int dy = -ry; dy <= ry; ++dy)
                            for (int dx = -rx; dx <= rx; ++dx) {
                                const int y = clampi(i + dy, 0, h - 1);
                                const long long r = ll[((size_t)b * h + y) * w + clampi(j + dx, 0, w - 1)];
                                const long long t = lr[((size_t)b * h + y) * w + clampi(j - d + dx, 0, w - 1)];
                                SR += r; SRR += r * r; ST += t; STT += t * t; SRT += r * t;
                            }
                        const long long N = n * SRT - SR * ST;
                        const long long A = n * SRR - SR * SR, Bv = n * STT - ST * ST;
                        if (A == 0 || Bv == 0)
                            C = 1.0;
                        else
                            C = 1.0 - (double)N / sqrt((double)A * (double)Bv);
                    }
                    out[(((size_t)b * h + i) * w + j) * D + d] = (int32_t)floor(32.0 * C + 0.5);
                }
}

/* 3 x 3 median filter of a uint8 map, borders replicated. */
void or_median3(const uint8_t *in, int B, int h, int w, uint8_t *out)
{
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < w; ++j) {
                int v[9], n = 0;
                for (int u = -1; u <= 1; ++u)
                    for (int t = -1; t <= 1; ++t)
                        v[n++] = in[((size_t)b * h + clampi(i + u, 0, h - 1)) * w + clampi(j + t, 0, w - 1)];
                /* insertion sort, then the middle element */
                for (int a = 1; a < 9; ++a)
                    for (int c = a; c > 0 && v[c - 1] > v[c]; --c) {
                        int tmp = v[c];
                        v[c] = v[c - 1];
                        v[c - 1] = tmp;
                    }
                out[((size_t)b * h + i) * w + j] = (uint8_t)v[4];
            }
}

/* ------------------------------------------------------------------------ */
/* Network primitives (Table I), FP64, NCHW.                                 */
/* ------------------------------------------------------------------------ */

/* 2-D convolution (cross-correlation), zero padding:
 *   y[b,o,p,q] = bias[o] + sum_{c,u,v} wt[o,c,u,v] * x[b,c, s*p+u-pad, s*q+v-pad]
 * Output size Ho = (H + 2*pad - k)/s + 1. */
void or_conv2d(const double *x, int B, int C, int H, int W, const double *wt, const double *bias,
               int O, int k, int s, int pad, double *y)
{
    int Ho = (H + 2 * pad - k) / s + 1, Wo = (W + 2 * pad - k) / s + 1;
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < O; ++o)
            for (int p = 0; p < Ho; ++p)
                for (int q = 0; q < Wo; ++q) {
                    double acc = bias ? bias[o] : 0.0;
                    for (int c = 0; c < C; ++c)
                        for (int u = 0; u < k; ++u)
                            for (int v = 0; v < k; ++v) {
                                int yy = s * p + u - pad, xx = s * q + v - pad;
                                if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                                    continue;
                                acc += wt[(((size_t)o * C + c) * k + u) * k + v] *
                                       x[(((size_t)b * C + c) * H + yy) * W + xx];
                            }
                    y[(((size_t)b * O + o) * Ho + p) * Wo + q] = acc;
                }
}

/* Adjoint of or_conv2d with respect to x: every term of the forward sum that
 * reads x[...] sends wt * dy back to it.  dx is overwritten. */
void or_conv2d_dx(const double *dy, int B, int C, int H, int W, const double *wt, int O, int k,
                  int s, int pad, double *dx)
{
    int Ho = (H + 2 * pad - k) / s + 1, Wo = (W + 2 * pad - k) / s + 1;
    memset(dx, 0, sizeof(double) * (size_t)B * C * H * W);
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < O; ++o)
            for (int p = 0; p < Ho; ++p)
                for (int q = 0; q < Wo; ++q) {
                    double g = dy[(((size_t)b * O + o) * Ho + p) * Wo + q];
                    for (int c = 0; c < C; ++c)
                        for (int u = 0; u < k; ++u)
                            for (int v = 0; v < k; ++v) {
                                int yy = s * p + u - pad, xx = s * q + v - pad;
                                if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                                    continue;
                                dx[(((size_t)b * C + c) * H + yy) * W + xx] +=
                                    wt[(((size_t)o * C + c) * k + u) * k + v] * g;
                            }
                }
}

/* Adjoint of or_conv2d with respect to wt and bias (overwritten). */
void or_conv2d_dw(const double *x, const double *dy, int B, int C, int H, int W, int O, int k,
                  int s, int pad, double *dwt, double *dbias)
{
    int Ho = (H + 2 * pad - k) / s + 1, Wo = (W + 2 * pad - k) / s + 1;
    memset(dwt, 0, sizeof(double) * (size_t)O * C * k * k);
    if (dbias)
        memset(dbias, 0, sizeof(double) * (size_t)O);
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < O; ++o)
            for (int p = 0; p < Ho; ++p)
                for (int q = 0; q < Wo; ++q) {
                    double g = dy[(((size_t)b * O + o) * Ho + p) * Wo + q];
                    if (dbias)
                        dbias[o] += g;
                    for (int c = 0; c < C; ++c)
                        for (int u = 0; u < k; ++u)
                            for (int v = 0; v < k; ++v) {
                                int yy = s * p + u - pad, xx = s * q + v - pad;
                                if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                                    continue;
                                dwt[(((size_t)o * C + c) * k + u) * k + v] +=
                                    x[(((size_t)b * C + c) * H + yy) * W + xx] * g;
                            }
                }
}

/* Transposed 2-D convolution (the upsampling "deconvolution" layers of the
 * decoder and the final upsampling layer, Table I): every input sample
 * x[b,c,i,j] spreads over the output through the kernel placed at
 * (s*i - pad, s*j - pad):
 *   y[b,o,Y,X] = bias[o] + sum of wt[o,c,u,v] * x[b,c,i,j]
 *                over (c, i, j, u, v) with s*i + u - pad = Y, s*j + v - pad = X,
 * for 0 <= Y < Ho, 0 <= X < Wo; terms that land outside are dropped.  Weights
 * are [O][C][k][k] (output channel first).  y is overwritten. */
void or_tconv2d(const double *x, int B, int C, int H, int W, const double *wt, const double *bias,
                int O, int k, int s, int pad, int Ho, int Wo, double *y)
{
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < O; ++o)
            for (size_t e = 0; e < (size_t)Ho * Wo; ++e)
                y[((size_t)b * O + o) * Ho * Wo + e] = bias ? bias[o] : 0.0;
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < O; ++o)
            for (int c = 0; c < C; ++c)
                for (int i = 0; i < H; ++i)
                    for (int j = 0; j < W; ++j) {
                        double xv = x[(((size_t)b * C + c) * H + i) * W + j];
                        for (int u = 0; u < k; ++u)
                            for (int v = 0; v < k; ++v) {
                                int Y = s * i + u - pad, X = s * j + v - pad;
                                if (Y < 0 || Y >= Ho || X < 0 || X >= Wo)
                                    continue;
                                y[(((size_t)b * O + o) * Ho + Y) * Wo + X] +=
                                    wt[(((size_t)o * C + c) * k + u) * k + v] * xv;
                            }
                    }
}

/* Source index pair and weight of bilinear resampling along one axis
 * (half-pixel centres, no corner alignment): s = (o + 1/2) * n_in / n_out - 1/2,
 * clamped below at 0; i0 = floor(s), i1 = min(i0 + 1, n_in - 1), lambda = s - i0. */
static void bilinear_axis(int o, int n_in, int n_out, int *i0, int *i1, double *lam)
{
    double s = ((double)o + 0.5) * (double)n_in / (double)n_out - 0.5;
    if (s < 0.0)
        s = 0.0;
    int a = (int)floor(s);
    if (a > n_in - 1)
        a = n_in - 1;
    *i0 = a;
    *i1 = a + 1 < n_in ? a + 1 : n_in - 1;
    *lam = s - (double)a;
}

/* Bilinear resize of N planes from Hi x Wi to Ho x Wo (upsampling layers of
 * the decoder and the final upsampling layer, Table I):
 *   y[n,p,q] = sum over the 2x2 source neighbourhood of (1-ly|ly)(1-lx|lx) x[...] */
void or_resize_bilinear(const double *x, int N, int Hi, int Wi, int Ho, int Wo, double *y)
{
    for (int n = 0; n < N; ++n)
        for (int p = 0; p < Ho; ++p) {
            int y0, y1;
            double ly;
            bilinear_axis(p, Hi, Ho, &y0, &y1, &ly);
            for (int q = 0; q < Wo; ++q) {
                int x0, x1;
                double lx;
                bilinear_axis(q, Wi, Wo, &x0, &x1, &lx);
                const double *src = x + (size_t)n * Hi * Wi;
                double top = (1.0 - lx) * src[(size_t)y0 * Wi + x0] + lx * src[(size_t)y0 * Wi + x1];
                double bot = (1.0 - lx) * src[(size_t)y1 * Wi + x0] + lx * src[(size_t)y1 * Wi + x1];
                y[((size_t)n * Ho + p) * Wo + q] = (1.0 - ly) * top + ly * bot;
            }
        }
}

/* Adjoint of or_resize_bilinear: each output's gradient goes back to its four
 * sources with the same weights.  dx is overwritten. */
void or_resize_bilinear_adj(const double *dy, int N, int Hi, int Wi, int Ho, int Wo, double *dx)
{
    memset(dx, 0, sizeof(double) * (size_t)N * Hi * Wi);
    for (int n = 0; n < N; ++n)
        for (int p = 0; p < Ho; ++p) {
            int y0, y1;
            double ly;
            bilinear_axis(p, Hi, Ho, &y0, &y1, &ly);
            for (int q = 0; q < Wo; ++q) {
                int x0, x1;
                double lx;
                bilinear_axis(q, Wi, Wo, &x0, &x1, &lx);
                double g = dy[((size_t)n * Ho + p) * Wo + q];
                double *d = dx + (size_t)n * Hi * Wi;
                d[(size_t)y0 * Wi + x0] += (1.0 - ly) * (1.0 - lx) * g;
                d[(size_t)y0 * Wi + x1] += (1.0 - ly) * lx * g;
                d[(size_t)y1 * Wi + x0] += ly * (1.0 - lx) * g;
                d[(size_t)y1 * Wi + x1] += ly * lx * g;
            }
        }
}
