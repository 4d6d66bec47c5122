/*
 * CPU oracle for the SLIC superpixel path (Ren, Prisacariu and Reid, gSLICr,
 * arXiv 1509.04232).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, sequential, obviously
 * correct statement of what the GPU path must compute.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the GPU
 * library; each side derives its own constants from the definitions below.
 *
 * Arithmetic contract (both sides): FP32 with every + - * / sqrt rounded to
 * nearest-even, evaluated strictly in the order written here, no fused
 * multiply-add (build with -ffp-contract=off), no reassociation, denormals
 * kept.  Centre sums are exact integers, so summation order cannot matter.
 *
 * Paper map: Section 2 defines the 5-D [l a b x y] space, the grid interval
 * S = sqrt(N/K), the distance of Eq. 1, the lowest-gradient seed perturbation,
 * the local k-means and the final connectivity clean-up.  Section 3 fixes the
 * GPU structure (a maximum of nine candidate centres per pixel, one thread per
 * pixel or per cluster).  Section 4's listing fixes the control flow:
 * convert, initialise centres, associate, then n times (update, associate),
 * then optionally enforce connectivity.
 *
 * Readings where the paper is silent are marked READING and are collected
 * in the design notes of the repository.
 *
 * Threads: loops whose iterations are independent (one pixel, one cell)
 * are split over OpenMP threads when the file is built with -fopenmp; every
 * value is still computed by the same operations in the same order, and the
 * centre sums are exact integers, so results do not depend on the thread
 * count.  Sums in floating point (the energy) stay sequential.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

/* READING: fixed-point scale of the per-pixel colour values entering the
 * centre sums (Section 3, "Updating the cluster center").  q = rint(v * 2^18)
 * with |v| < 108 gives |q| < 2^25. */
#define ORC_QSHIFT 18

int orc_version(void) { return 1; }

/* Threads used by the parallel loops: n > 0 sets the count, n == 0 only
 * queries it; 1 without OpenMP. */
int orc_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
int orc_qshift(void) { return ORC_QSHIFT; }

/* ------------------------------------------------------------------------
 * O0. Grid (Section 2: a centre every S = sqrt(N/K) pixels; Section 3: an
 * ns_r x ns_c superpixel map).
 * READING: S is an integer.  Given K instead of S, S = floor(sqrt(N/K)+0.5),
 * at least 1.  Cells are S x S, the last row/column of cells may be partial:
 * ns_c = ceil(W/S), ns_r = ceil(H/S), cluster k = cy*ns_c + cx.
 * ---------------------------------------------------------------------- */
int orc_grid(int32_t w, int32_t h, int32_t S_in, int32_t K_in, int32_t* S_out,
             int32_t* ns_c, int32_t* ns_r) {
    if (w < 1 || h < 1) return ORC_EINVAL;
    int32_t S = S_in;
    if (S <= 0) {
        if (K_in <= 0) return ORC_EINVAL;
        double n = (double)w * (double)h;
        double s = floor(sqrt(n / (double)K_in) + 0.5);
        S = s < 1.0 ? 1 : (int32_t)s;
    }
    *S_out = S;
    *ns_c = (w + S - 1) / S;
    *ns_r = (h + S - 1) / S;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * O1. RGB -> CIELAB (Section 3: the input is converted to CIELAB, one thread
 * per pixel; Section 2: CIELAB is used because it is perceptually uniform).
 * READING: sRGB (IEC 61966-2-1) primaries and transfer curve, D65 white,
 * R,G,B byte order, FP32 output.
 * ---------------------------------------------------------------------- */

/* Cube root of t > 0 (normal).  t = f*2^e with f in [0.5,1); e is shifted
 * to a multiple of three so that g = f*2^r lies in [0.5,4) and
 * cbrt(t) = cbrt(g)*2^q.  Newton's method on the inverse cube root,
 * y <- y + y(1 - g y^3)/3, needs no division; a quadratic seed on [0.5,4)
 * has relative error below 4.2%, each step squares the error, so four steps
 * reach the double-precision fixed point.  Then cbrt(g) = g*y*y, within
 * three ulps of the true root; cbrt(1) is exactly 1. */
static double orc_cbrt(double t) {
    int e;
    double f = frexp(t, &e);
    int r = ((e % 3) + 3) % 3;
    double g = ldexp(f, r);
    int q = (e - r) / 3;
    double lin = 1.405 - 0.4258 * g;
    double g2 = g * g;
    double y = lin + 0.05965 * g2;
    const double third = 1.0 / 3.0;
    for (int i = 0; i < 4; i++) {
        double y2 = y * y;
        double y3 = y2 * y;
        double err = fma(-g, y3, 1.0);
        double corr = y * err;
        y = fma(corr, third, y);
    }
    double c = g * y;
    c = c * y;
    return ldexp(c, q);
}

double orc_cbrt_export(double t) { return orc_cbrt(t); }

/* 256-entry sRGB decode table and the XYZ matrix with each row divided by
 * its sum, so that X/Xn, Y/Yn, Z/Zn come out directly (D65 white = the row
 * sums 0.9505, 1.0, 1.089). */
void orc_lab_tables(float lin[256], float nmat[9]) {
    for (int v = 0; v < 256; v++) {
        double c = (double)v / 255.0;
        double l = c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
        lin[v] = (float)l;
    }
    static const double M[3][3] = {{0.4124, 0.3576, 0.1805},
                                   {0.2126, 0.7152, 0.0722},
                                   {0.0193, 0.1192, 0.9505}};
    for (int i = 0; i < 3; i++) {
        double rs = (M[i][0] + M[i][1]) + M[i][2];
        for (int j = 0; j < 3; j++) nmat[3 * i + j] = (float)(M[i][j] / rs);
    }
}

/* CIE f(t): cube root above (6/29)^3 = 216/24389, the linear segment
 * (24389/27 * t + 16)/116 below; evaluated in FP64, rounded to FP32. */
static float orc_lab_f(float t) {
    double td = (double)t;
    double eps = 216.0 / 24389.0;
    double kap = 24389.0 / 27.0;
    double r;
    if (td > eps) {
        r = orc_cbrt(td);
    } else {
        double p = kap * td;
        double s = p + 16.0;
        r = s / 116.0;
    }
    return (float)r;
}

int orc_rgb_to_lab(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch, int32_t channels,
                   float* L, float* A, float* B) {
    if (!rgb || !L || !A || !B || w < 1 || h < 1 || (channels != 3 && channels != 4) ||
        pitch < w * channels)
        return ORC_EINVAL;
    float lin[256], nm[9];
    orc_lab_tables(lin, nm);
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < h; y++) {
        for (int32_t x = 0; x < w; x++) {
            const uint8_t* p = rgb + (size_t)y * pitch + (size_t)x * channels;
            float r = lin[p[0]], g = lin[p[1]], b = lin[p[2]];
            float X = nm[0] * r;
            X = X + nm[1] * g;
            X = X + nm[2] * b;
            float Y = nm[3] * r;
            Y = Y + nm[4] * g;
            Y = Y + nm[5] * b;
            float Z = nm[6] * r;
            Z = Z + nm[7] * g;
            Z = Z + nm[8] * b;
            float fx = orc_lab_f(X), fy = orc_lab_f(Y), fz = orc_lab_f(Z);
            size_t i = (size_t)y * w + x;
            float l = 116.0f * fy;
            L[i] = l - 16.0f;
            float dxy = fx - fy;
            A[i] = 500.0f * dxy;
            float dyz = fy - fz;
            B[i] = 200.0f * dyz;
        }
    }
    return ORC_OK;
}

/* Other colour spaces (the listing's colour_space setting; the paper
 * describes only CIELAB).  READING: space 1 is XYZ scaled by 100 (D65 white
 * -> (100, 100, 100) with the row-normalised matrix above), computed in FP32
 * in the order of the Lab path and then multiplied by 100; space 2 is the
 * raw R, G, B bytes as floats.  Space 0 is CIELAB. */
int orc_rgb_to_space(const uint8_t* rgb, int32_t w, int32_t h, int32_t pitch, int32_t channels,
                     int32_t space, float* C0, float* C1, float* C2) {
    if (space == 0) return orc_rgb_to_lab(rgb, w, h, pitch, channels, C0, C1, C2);
    if (!rgb || !C0 || !C1 || !C2 || w < 1 || h < 1 || (channels != 3 && channels != 4) ||
        pitch < w * channels || (space != 1 && space != 2))
        return ORC_EINVAL;
    float lin[256], nm[9];
    orc_lab_tables(lin, nm);
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < h; y++) {
        for (int32_t x = 0; x < w; x++) {
            const uint8_t* p = rgb + (size_t)y * pitch + (size_t)x * channels;
            size_t i = (size_t)y * w + x;
            if (space == 2) {
                C0[i] = (float)p[0];
                C1[i] = (float)p[1];
                C2[i] = (float)p[2];
                continue;
            }
            float r = lin[p[0]], g = lin[p[1]], b = lin[p[2]];
            float X = nm[0] * r;
            X = X + nm[1] * g;
            X = X + nm[2] * b;
            float Y = nm[3] * r;
            Y = Y + nm[4] * g;
            Y = Y + nm[5] * b;
            float Z = nm[6] * r;
            Z = Z + nm[7] * g;
            Z = Z + nm[8] * b;
            C0[i] = 100.0f * X;
            C1[i] = 100.0f * Y;
            C2[i] = 100.0f * Z;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * O2. Seeds (Section 2: centres on the S grid, perturbed to the lowest
 * gradient position in a local neighbourhood; Section 3: one thread per
 * centre fills the superpixel map).
 * READING: the gradient is the one of the cited SLIC paper,
 *   G(x,y) = |I(x+1,y) - I(x-1,y)|^2 + |I(x,y+1) - I(x,y-1)|^2
 * over the Lab vector I, with coordinates clamped to the image.  The seed of
 * cell (cx,cy) is its middle pixel x0 + (x1-x0-1)/2; the neighbourhood is the
 * 3x3 window around it, scanned row by row, moving only on a strictly
 * smaller gradient.  The centre takes the chosen pixel's Lab and position.
 * ---------------------------------------------------------------------- */
static float orc_sq3(float u, float v, float s) {
    float a = u * u;
    a = a + v * v;
    a = a + s * s;
    return a;
}

static float orc_gradient(const float* L, const float* A, const float* B, int32_t w, int32_t h,
                          int32_t x, int32_t y) {
    int32_t xl = x > 0 ? x - 1 : 0, xr = x < w - 1 ? x + 1 : w - 1;
    int32_t yu = y > 0 ? y - 1 : 0, yd = y < h - 1 ? y + 1 : h - 1;
    size_t r = (size_t)y * w, c = (size_t)x;
    float gx = orc_sq3(L[r + xr] - L[r + xl], A[r + xr] - A[r + xl], B[r + xr] - B[r + xl]);
    size_t u = (size_t)yu * w + c, d = (size_t)yd * w + c;
    float gy = orc_sq3(L[d] - L[u], A[d] - A[u], B[d] - B[u]);
    return gx + gy;
}

float orc_gradient_at(const float* L, const float* A, const float* B, int32_t w, int32_t h,
                      int32_t x, int32_t y) {
    return orc_gradient(L, A, B, w, h, x, y);
}

/* centres: K x 5 floats (L, a, b, x, y) */
int orc_seed(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
             int32_t perturb, float* centres) {
    if (!L || !A || !B || !centres || w < 1 || h < 1 || S < 1) return ORC_EINVAL;
    int32_t ns_c = (w + S - 1) / S, ns_r = (h + S - 1) / S;
#pragma omp parallel for schedule(static)
    for (int32_t cy = 0; cy < ns_r; cy++) {
        for (int32_t cx = 0; cx < ns_c; cx++) {
            int32_t x0 = cx * S, x1 = x0 + S < w ? x0 + S : w;
            int32_t y0 = cy * S, y1 = y0 + S < h ? y0 + S : h;
            int32_t sx = x0 + (x1 - x0 - 1) / 2, sy = y0 + (y1 - y0 - 1) / 2;
            int32_t bx = sx, by = sy;
            if (perturb) {
                float gbest = orc_gradient(L, A, B, w, h, sx, sy);
                for (int32_t dy = -1; dy <= 1; dy++) {
                    for (int32_t dx = -1; dx <= 1; dx++) {
                        int32_t nx = sx + dx, ny = sy + dy;
                        if (nx < 0 || nx >= w || ny < 0 || ny >= h) continue;
                        float g = orc_gradient(L, A, B, w, h, nx, ny);
                        if (g < gbest) {
                            gbest = g;
                            bx = nx;
                            by = ny;
                        }
                    }
                }
            }
            size_t i = (size_t)by * w + bx;
            float* c = centres + 5 * ((size_t)cy * ns_c + cx);
            c[0] = L[i];
            c[1] = A[i];
            c[2] = B[i];
            c[3] = (float)bx;
            c[4] = (float)by;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * O3. Association (Eq. 1 and Section 3, "Finding the cluster associations"):
 *   d_lab = sqrt(dl^2 + da^2 + db^2), d_xy = sqrt(dx^2 + dy^2),
 *   D_s = d_lab + (m/S) d_xy
 * (the third term of d_lab subtracts the b components; the equation's n_k is
 * a misprint of b_k).  The candidates are the centres of the pixel's own
 * grid cell and its eight neighbours, the "maximum of nine" of Section 3.
 * READING: ties go to the lowest cluster index (candidates are visited in
 * increasing index and replaced only on a strictly smaller distance).
 * ---------------------------------------------------------------------- */
static float orc_distance(const float* c, float l, float a, float b, int32_t x, int32_t y,
                          float wgt) {
    float dl = c[0] - l, da = c[1] - a, db = c[2] - b;
    float dlab = sqrtf(orc_sq3(dl, da, db));
    float dx = c[3] - (float)x, dy = c[4] - (float)y;
    float s = dx * dx;
    s = s + dy * dy;
    float dxy = sqrtf(s);
    float sp = wgt * dxy;
    return dlab + sp;
}

/* The distance of the SLIC paper the method builds on, as an option:
 * D^2 = d_lab^2 + (m/S)^2 d_xy^2 (the argmin of its square root), in FP32 in
 * this order without square roots; its energy term is sqrt(D^2). */
static float orc_distance_sq(const float* c, float l, float a, float b, int32_t x, int32_t y,
                             float wgt) {
    float dl = c[0] - l, da = c[1] - a, db = c[2] - b;
    float s = orc_sq3(dl, da, db);
    float dx = c[3] - (float)x, dy = c[4] - (float)y;
    float t = dx * dx;
    t = t + dy * dy;
    float w2 = wgt * wgt;
    float sp = w2 * t;
    return s + sp;
}

static float orc_dist(int32_t dist, const float* c, float l, float a, float b, int32_t x,
                      int32_t y, float wgt) {
    return dist ? orc_distance_sq(c, l, a, b, x, y, wgt) : orc_distance(c, l, a, b, x, y, wgt);
}

float orc_weight(float m, int32_t S) { return m / (float)S; }

int orc_assign_ex(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
                  float m, int32_t dist, const float* centres, int32_t* labels) {
    if (!L || !A || !B || !centres || !labels || w < 1 || h < 1 || S < 1) return ORC_EINVAL;
    int32_t ns_c = (w + S - 1) / S, ns_r = (h + S - 1) / S;
    float wgt = orc_weight(m, S);
#pragma omp parallel for schedule(static)
    for (int32_t y = 0; y < h; y++) {
        for (int32_t x = 0; x < w; x++) {
            size_t i = (size_t)y * w + x;
            int32_t gx = x / S, gy = y / S;
            int32_t bk = -1;
            float best = 0.0f;
            for (int32_t dy = -1; dy <= 1; dy++) {
                int32_t cy = gy + dy;
                if (cy < 0 || cy >= ns_r) continue;
                for (int32_t dx = -1; dx <= 1; dx++) {
                    int32_t cx = gx + dx;
                    if (cx < 0 || cx >= ns_c) continue;
                    int32_t k = cy * ns_c + cx;
                    float d = orc_dist(dist, centres + 5 * (size_t)k, L[i], A[i], B[i], x, y, wgt);
                    if (bk < 0 || d < best) {
                        best = d;
                        bk = k;
                    }
                }
            }
            labels[i] = bk;
        }
    }
    return ORC_OK;
}

int orc_assign(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
               float m, const float* centres, int32_t* labels) {
    return orc_assign_ex(L, A, B, w, h, S, m, 0, centres, labels);
}

/* ------------------------------------------------------------------------
 * O4. Centre update (Section 2: new centre locations; Section 3, "Updating
 * the cluster center": each centre gathers the pixels associated with it).
 * The new centre is the mean of its pixels' [l a b x y].
 * READING: colour values enter the sums as exact integers q = rint(v*2^18)
 * (round half to even); x, y are integers already.  Sums are int64, so any
 * order of summation gives the same result.  The mean is the FP64 quotient
 * sum/count, scaled back by 2^-18 and rounded to FP32.  A centre with no
 * pixels keeps its previous value.  votes: NULL, or only the pixels with
 * votes[i] != 0 are counted (the learned warm start's first update takes
 * its confident pixels this way); every label must still be a cluster.
 * ---------------------------------------------------------------------- */
int orc_update_votes(const float* L, const float* A, const float* B, int32_t w, int32_t h,
                     const int32_t* labels, const uint8_t* votes, int32_t K, float* centres,
                     int32_t* counts) {
    if (!L || !A || !B || !labels || !centres || !counts || w < 1 || h < 1 || K < 1)
        return ORC_EINVAL;
    for (size_t i = 0; i < (size_t)w * h; i++)
        if (labels[i] < 0 || labels[i] >= K) return ORC_EINVAL;
    /* sums[k] = (sum qL, sum qa, sum qb, sum x, sum y, count) */
    int64_t* sums = (int64_t*)calloc((size_t)K * 6, sizeof(int64_t));
    if (!sums) return ORC_ENOMEM;
    const float scale = (float)(1 << ORC_QSHIFT);
    int failed = 0;
    /* each thread adds its rows into sums of its own, then into the total;
     * integer additions give the same total in any order */
#pragma omp parallel
    {
        int64_t* part = (int64_t*)calloc((size_t)K * 6, sizeof(int64_t));
        if (!part) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int32_t y = 0; y < h; y++) {
            if (!part) continue;
            for (int32_t x = 0; x < w; x++) {
                size_t i = (size_t)y * w + x;
                int32_t k = labels[i];
                if (votes && !votes[i]) continue;
                int64_t* s = part + 6 * (size_t)k;
                s[0] += llrintf(L[i] * scale);
                s[1] += llrintf(A[i] * scale);
                s[2] += llrintf(B[i] * scale);
                s[3] += x;
                s[4] += y;
                s[5] += 1;
            }
        }
        if (part) {
#pragma omp critical
            for (size_t j = 0; j < (size_t)K * 6; j++) sums[j] += part[j];
            free(part);
        }
    }
    if (failed) {
        free(sums);
        return ORC_ENOMEM;
    }
    const double inv = 1.0 / (double)(1 << ORC_QSHIFT);
    for (int32_t k = 0; k < K; k++) counts[k] = (int32_t)sums[6 * (size_t)k + 5];
    for (int32_t k = 0; k < K; k++) {
        if (counts[k] == 0) continue;
        double n = (double)counts[k];
        int64_t* s = sums + 6 * (size_t)k;
        float* c = centres + 5 * (size_t)k;
        for (int j = 0; j < 3; j++) {
            double mean = (double)s[j] / n;
            c[j] = (float)(mean * inv);
        }
        c[3] = (float)((double)s[3] / n);
        c[4] = (float)((double)s[4] / n);
    }
    free(sums);
    return ORC_OK;
}

int orc_update(const float* L, const float* A, const float* B, int32_t w, int32_t h,
               const int32_t* labels, int32_t K, float* centres, int32_t* counts) {
    return orc_update_votes(L, A, B, w, h, labels, NULL, K, centres, counts);
}

/* ------------------------------------------------------------------------
 * O5. The loop of Section 4's listing: convert, seed, associate, then
 * `iters` times (update, associate).  The returned centres are those the
 * last association used; counts are those of the last update (zero when
 * iters == 0).  READING: a fixed iteration count; the L1 stopping threshold
 * of Section 2 is a separate option.
 * ---------------------------------------------------------------------- */
int orc_kmeans_ex(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
                  float m, int32_t dist, int32_t perturb, int32_t iters, float* centres,
                  int32_t* counts, int32_t* labels) {
    if (w < 1 || h < 1 || S < 1 || iters < 0) return ORC_EINVAL;
    int32_t K = ((w + S - 1) / S) * ((h + S - 1) / S);
    int rc = orc_seed(L, A, B, w, h, S, perturb, centres);
    if (rc) return rc;
    for (int32_t k = 0; k < K; k++) counts[k] = 0;
    rc = orc_assign_ex(L, A, B, w, h, S, m, dist, centres, labels);
    if (rc) return rc;
    for (int32_t it = 0; it < iters; it++) {
        rc = orc_update(L, A, B, w, h, labels, K, centres, counts);
        if (rc) return rc;
        rc = orc_assign_ex(L, A, B, w, h, S, m, dist, centres, labels);
        if (rc) return rc;
    }
    return ORC_OK;
}

int orc_kmeans(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
               float m, int32_t perturb, int32_t iters, float* centres, int32_t* counts,
               int32_t* labels) {
    return orc_kmeans_ex(L, A, B, w, h, S, m, 0, perturb, iters, centres, counts, labels);
}

/* ------------------------------------------------------------------------
 * Convergence stop (Section 2 ends the loop once the centres move by less
 * than a threshold in L1 from one iteration to the next).
 * READING: the distance is summed over every centre and its five components
 * (L, a, b, x, y), each |difference| taken in FP64 and quantised to
 * rint(|d| * 2^18) so that the sum is an exact integer; the threshold T is
 * the mean shift per centre, so the loop stops after the first iteration i
 * (update, then association) whose sum is below rint(T * 2^18) * K.  At most
 * max_iters iterations; *iters_done receives the number run.
 * ---------------------------------------------------------------------- */
int64_t orc_residual(const float* prev, const float* next, int32_t K) {
    int64_t r = 0;
    for (size_t i = 0; i < (size_t)K * 5; i++)
        r += llrint(fabs((double)next[i] - (double)prev[i]) * (double)(1 << ORC_QSHIFT));
    return r;
}

int orc_kmeans_converge(const float* L, const float* A, const float* B, int32_t w, int32_t h,
                        int32_t S, float m, int32_t perturb, int32_t max_iters, float threshold,
                        float* centres, int32_t* counts, int32_t* labels, int32_t* iters_done) {
    if (w < 1 || h < 1 || S < 1 || max_iters < 0 || !iters_done || !(threshold >= 0.0f))
        return ORC_EINVAL;
    int32_t K = ((w + S - 1) / S) * ((h + S - 1) / S);
    const int64_t limit = llrint((double)threshold * (double)(1 << ORC_QSHIFT)) * (int64_t)K;
    float* prev = malloc(sizeof(float) * 5 * (size_t)K);
    if (!prev) return ORC_ENOMEM;
    int rc = orc_seed(L, A, B, w, h, S, perturb, centres);
    for (int32_t k = 0; !rc && k < K; k++) counts[k] = 0;
    if (!rc) rc = orc_assign(L, A, B, w, h, S, m, centres, labels);
    *iters_done = 0;
    for (int32_t it = 0; !rc && it < max_iters; it++) {
        memcpy(prev, centres, sizeof(float) * 5 * (size_t)K);
        rc = orc_update(L, A, B, w, h, labels, K, centres, counts);
        if (!rc) rc = orc_assign(L, A, B, w, h, S, m, centres, labels);
        if (rc) break;
        *iters_done = it + 1;
        if (orc_residual(prev, centres, K) < limit) break;
    }
    free(prev);
    return rc;
}

/* ------------------------------------------------------------------------
 * O7. Energy: the mean over pixels of Eq. 1's D_s between each pixel and the
 * centre it is associated with, each term computed exactly as in O3 and
 * summed in FP64 in raster order.
 * ---------------------------------------------------------------------- */
int orc_energy_ex(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
                  float m, int32_t dist, const float* centres, int32_t K, const int32_t* labels,
                  double* out) {
    if (!L || !A || !B || !centres || !labels || !out || w < 1 || h < 1 || S < 1) return ORC_EINVAL;
    float wgt = orc_weight(m, S);
    double acc = 0.0;
    for (int32_t y = 0; y < h; y++) {
        for (int32_t x = 0; x < w; x++) {
            size_t i = (size_t)y * w + x;
            int32_t k = labels[i];
            if (k < 0 || k >= K) return ORC_EINVAL;
            float d = orc_dist(dist, centres + 5 * (size_t)k, L[i], A[i], B[i], x, y, wgt);
            acc += (double)(dist ? sqrtf(d) : d);
        }
    }
    *out = acc / ((double)w * (double)h);
    return ORC_OK;
}

int orc_energy(const float* L, const float* A, const float* B, int32_t w, int32_t h, int32_t S,
               float m, const float* centres, int32_t K, const int32_t* labels, double* out) {
    return orc_energy_ex(L, A, B, w, h, S, m, 0, centres, K, labels, out);
}

/* ------------------------------------------------------------------------
 * O6. Connectivity (Section 2: connectivity is enforced to clean up the
 * final lattice).  READING, a canonical merge rule:
 *  1. 4-connected components of equal label; a component is named by its
 *     smallest raster index (its root pixel r);
 *  2. a component is small if size < min_segment (min_segment > 0) or
 *     4*size < S*S (min_segment == 0);
 *  3. every small component other than the one holding pixel 0 joins the
 *     component of the pixel left of r (or above r when r starts a row);
 *     that pixel precedes r, so the joins form a forest;
 *  4. each component takes its tree root's segment; segments are numbered
 *     0.. in raster order of their roots (= order of first appearance).
 * seg_cluster[s] (optional) receives the input label of segment s's root.
 * ---------------------------------------------------------------------- */
int orc_connectivity(const int32_t* labels, int32_t w, int32_t h, int32_t S, int32_t min_segment,
                     int32_t* out, int32_t* n_segments, int32_t* seg_cluster) {
    if (!labels || !out || !n_segments || w < 1 || h < 1 || S < 1 || min_segment < 0)
        return ORC_EINVAL;
    size_t n = (size_t)w * h;
    int32_t* comp = (int32_t*)malloc(n * sizeof(int32_t));
    int32_t* size = (int32_t*)calloc(n, sizeof(int32_t));
    int32_t* stack = (int32_t*)malloc(n * sizeof(int32_t));
    int32_t* join = (int32_t*)malloc(n * sizeof(int32_t));
    int32_t* rank = (int32_t*)malloc(n * sizeof(int32_t));
    if (!comp || !size || !stack || !join || !rank) {
        free(comp); free(size); free(stack); free(join); free(rank);
        return ORC_ENOMEM;
    }
    for (size_t i = 0; i < n; i++) comp[i] = -1;
    /* 1. flood fill from each unvisited pixel in raster order */
    for (size_t r = 0; r < n; r++) {
        if (comp[r] >= 0) continue;
        int32_t lab = labels[r];
        size_t top = 0;
        stack[top++] = (int32_t)r;
        comp[r] = (int32_t)r;
        while (top > 0) {
            int32_t p = stack[--top];
            size[r] += 1;
            int32_t px = p % w, py = p / w;
            int32_t nb[4] = {px > 0 ? p - 1 : -1, px < w - 1 ? p + 1 : -1, py > 0 ? p - w : -1,
                             py < h - 1 ? p + w : -1};
            for (int j = 0; j < 4; j++) {
                int32_t q = nb[j];
                if (q >= 0 && comp[q] < 0 && labels[q] == lab) {
                    comp[q] = (int32_t)r;
                    stack[top++] = q;
                }
            }
        }
    }
    /* 2.-3. joins of small components, resolved in raster order (a join
     * always points to an earlier root, which is already resolved) */
    for (size_t r = 0; r < n; r++) {
        if (comp[r] != (int32_t)r) continue;
        int small = min_segment > 0 ? size[r] < min_segment
                                    : (int64_t)4 * size[r] < (int64_t)S * (int64_t)S;
        if (r != 0 && small) {
            int32_t x = (int32_t)(r % (size_t)w);
            size_t q = x > 0 ? r - 1 : r - (size_t)w;
            join[r] = join[comp[q]];
        } else {
            join[r] = (int32_t)r;
        }
    }
    /* 4. number the surviving roots in raster order */
    int32_t ns = 0;
    for (size_t r = 0; r < n; r++) {
        if (comp[r] == (int32_t)r && join[r] == (int32_t)r) {
            if (seg_cluster) seg_cluster[ns] = labels[r];
            rank[r] = ns++;
        }
    }
    for (size_t i = 0; i < n; i++) out[i] = rank[join[comp[i]]];
    *n_segments = ns;
    free(comp); free(size); free(stack); free(join); free(rank);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Stray-pixel filter (Section 3's clean-up step: a pixel whose neighbours
 * all carry other labels adopts theirs; the same per-pixel pass runs twice).
 * READING: the neighbours are the 4-connected ones inside the
 * image (up, left, right, down).  A pixel none of whose neighbours shares its
 * label takes the label that occurs most often among them, ties going to the
 * first in the order up, left, right, down; every pixel decides from the
 * input of the pass (a pass reads one map and writes another).  `passes`
 * passes; in and out may not overlap.
 * ---------------------------------------------------------------------- */
static int32_t orc_stray_pixel(const int32_t* in, int32_t w, int32_t h, int32_t x, int32_t y) {
    const int32_t own = in[(size_t)y * w + x];
    int32_t nb[4];
    int n = 0;
    if (y > 0) nb[n++] = in[(size_t)(y - 1) * w + x];
    if (x > 0) nb[n++] = in[(size_t)y * w + x - 1];
    if (x + 1 < w) nb[n++] = in[(size_t)y * w + x + 1];
    if (y + 1 < h) nb[n++] = in[(size_t)(y + 1) * w + x];
    if (n == 0) return own;
    for (int i = 0; i < n; i++)
        if (nb[i] == own) return own;
    int best = 0, best_count = 0;
    for (int i = 0; i < n; i++) {
        int count = 0;
        for (int j = 0; j < n; j++) count += nb[j] == nb[i];
        if (count > best_count) {  /* strictly more: ties keep the earlier */
            best_count = count;
            best = i;
        }
    }
    return nb[best];
}

int orc_stray_filter(const int32_t* in, int32_t w, int32_t h, int32_t passes, int32_t* out) {
    if (!in || !out || w < 1 || h < 1 || passes < 0) return ORC_EINVAL;
    size_t n = (size_t)w * h;
    int32_t* tmp = malloc(sizeof(int32_t) * n);
    if (!tmp) return ORC_ENOMEM;
    memcpy(out, in, sizeof(int32_t) * n);
    for (int32_t p = 0; p < passes; p++) {
        memcpy(tmp, out, sizeof(int32_t) * n);
        for (int32_t y = 0; y < h; y++)
            for (int32_t x = 0; x < w; x++) out[(size_t)y * w + x] = orc_stray_pixel(tmp, w, h, x, y);
    }
    free(tmp);
    return ORC_OK;
}
