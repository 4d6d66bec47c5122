/*
 * Seeded synthetic test images for the SLIC superpixel path.
 *
 * The paper times its method on five unnamed photographs (Table 1) that are
 * not available; these piecewise-smooth images stand in for them.  An image
 * is a Voronoi partition of the frame into `regions` cells, each painted with
 * a uniform random base colour plus a linear ramp of +-`ramp` levels along a
 * random direction, plus i.i.d. Gaussian noise of standard deviation `sigma`,
 * rounded half-to-even and clamped to 0..255.
 *
 * This module holds none of the segmentation method's arithmetic; it only
 * produces the bytes that both the CPU oracle and the GPU path consume.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Its n-th output is a pure
 * function of (key, n), so the noise field is counter-based and the result
 * does not depend on how many threads fill the image.  Gaussian deviates use
 * the Box-Muller transform (cosine branch).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* n-th output (n >= 0) of the SplitMix64 stream started at `key`. */
static uint64_t sm_at(uint64_t key, uint64_t n) { return sm_mix(key + (n + 1) * SM_GAMMA); }

/* uniform double in [0, 1) with 53 random bits */
static double u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    uint64_t key;
    uint64_t n;
} sm_stream;

static uint64_t sm_next(sm_stream* s) { return sm_at(s->key, s->n++); }

/* Independent stream keys for the site positions, region styling and noise. */
static uint64_t stream_key(uint64_t seed, uint64_t domain) {
    return sm_mix(seed * 0xD1B54A32D192ED03ULL + domain * SM_GAMMA + 0x2545F4914F6CDD1DULL);
}

int synth_version(void) { return 1; }

/*
 * Fill `out` (h rows of w*3 bytes, R,G,B) with the image for `seed`; if
 * `region_out` is not NULL it receives each pixel's Voronoi region index.
 * Returns 0 on success, 1 on bad arguments, 2 on allocation failure.
 */
int synth_voronoi(uint8_t* out, int32_t* region_out, int32_t w, int32_t h, int32_t regions,
                  double ramp, double sigma, uint64_t seed) {
    if (!out || w < 1 || h < 1 || regions < 1 || !(ramp >= 0.0) || !(sigma >= 0.0)) return 1;
    const int n = regions;
    double* sx = (double*)malloc(sizeof(double) * n);
    double* sy = (double*)malloc(sizeof(double) * n);
    double* base = (double*)malloc(sizeof(double) * 3 * n);
    double* amp = (double*)malloc(sizeof(double) * 3 * n);
    double* ct = (double*)malloc(sizeof(double) * n);
    double* st = (double*)malloc(sizeof(double) * n);
    if (!sx || !sy || !base || !amp || !ct || !st) {
        free(sx); free(sy); free(base); free(amp); free(ct); free(st);
        return 2;
    }
    sm_stream site = {stream_key(seed, 1), 0};
    for (int i = 0; i < n; i++) {
        sx[i] = u01(sm_next(&site)) * (double)w;
        sy[i] = u01(sm_next(&site)) * (double)h;
    }
    sm_stream sty = {stream_key(seed, 2), 0};
    const double two_pi = 6.283185307179586476925286766559;
    for (int i = 0; i < n; i++) {
        for (int c = 0; c < 3; c++) base[3 * i + c] = (double)(sm_next(&sty) >> 56);
        double th = u01(sm_next(&sty)) * two_pi;
        ct[i] = cos(th);
        st[i] = sin(th);
        for (int c = 0; c < 3; c++) amp[3 * i + c] = (2.0 * u01(sm_next(&sty)) - 1.0) * ramp;
    }
    const double R = sqrt((double)w * (double)h / (3.14159265358979323846 * (double)n));

    /* Bucket grid over the sites for an exact nearest-site search. */
    double B = R > 1.0 ? R : 1.0;
    int gw = (int)ceil((double)w / B), gh = (int)ceil((double)h / B);
    if (gw < 1) gw = 1;
    if (gh < 1) gh = 1;
    int* bstart = (int*)calloc((size_t)gw * gh + 1, sizeof(int));
    int* bidx = (int*)malloc(sizeof(int) * n);
    int* bfill = (int*)calloc((size_t)gw * gh, sizeof(int));
    if (!bstart || !bidx || !bfill) {
        free(sx); free(sy); free(base); free(amp); free(ct); free(st);
        free(bstart); free(bidx); free(bfill);
        return 2;
    }
    for (int i = 0; i < n; i++) {
        int bx = (int)(sx[i] / B), by = (int)(sy[i] / B);
        if (bx >= gw) bx = gw - 1;
        if (by >= gh) by = gh - 1;
        bstart[by * gw + bx + 1]++;
    }
    for (int b = 0; b < gw * gh; b++) bstart[b + 1] += bstart[b];
    for (int i = 0; i < n; i++) { /* ascending site index inside each bucket */
        int bx = (int)(sx[i] / B), by = (int)(sy[i] / B);
        if (bx >= gw) bx = gw - 1;
        if (by >= gh) by = gh - 1;
        int b = by * gw + bx;
        bidx[bstart[b] + bfill[b]++] = i;
    }
    const uint64_t nkey = stream_key(seed, 3);
    const int gmax = gw > gh ? gw : gh;

#pragma omp parallel for schedule(static)
    for (int y = 0; y < h; y++) {
        int by = (int)((double)y / B);
        if (by >= gh) by = gh - 1;
        for (int x = 0; x < w; x++) {
            int bx = (int)((double)x / B);
            if (bx >= gw) bx = gw - 1;
            /* nearest site, ties to the lowest index; ring r of buckets is
             * searched until no site beyond it can be as close */
            double best = INFINITY;
            int bi = -1;
            for (int r = 0; r <= gmax; r++) {
                if (bi >= 0) {
                    double lim = (double)(r - 1) * B;
                    if (r >= 1 && best < lim * lim) break;
                }
                for (int yy = by - r; yy <= by + r; yy++) {
                    if (yy < 0 || yy >= gh) continue;
                    int edge = (yy == by - r || yy == by + r);
                    for (int xx = bx - r; xx <= bx + r; xx += (edge ? 1 : 2 * r)) {
                        if (xx >= 0 && xx < gw) {
                            int b = yy * gw + xx;
                            for (int j = bstart[b]; j < bstart[b + 1]; j++) {
                                int i = bidx[j];
                                double dx = sx[i] - (double)x, dy = sy[i] - (double)y;
                                double d2 = dx * dx + dy * dy;
                                if (d2 < best || (d2 == best && i < bi)) {
                                    best = d2;
                                    bi = i;
                                }
                            }
                        }
                        if (r == 0) break;
                    }
                }
            }
            double t = ((double)x - sx[bi]) * ct[bi] + ((double)y - sy[bi]) * st[bi];
            t = R > 0.0 ? t / R : 0.0;
            if (t < -1.0) t = -1.0;
            if (t > 1.0) t = 1.0;
            if (region_out) region_out[(size_t)y * w + x] = bi;
            uint8_t* px = out + ((size_t)y * w + x) * 3;
            for (int c = 0; c < 3; c++) {
                uint64_t k = ((uint64_t)y * (uint64_t)w + (uint64_t)x) * 3u + (uint64_t)c;
                double g = 0.0;
                if (sigma > 0.0) {
                    double u1 = 1.0 - u01(sm_at(nkey, 2 * k)); /* (0, 1] */
                    double u2 = u01(sm_at(nkey, 2 * k + 1));
                    g = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
                }
                double v = nearbyint(base[3 * bi + c] + amp[3 * bi + c] * t + sigma * g);
                if (v < 0.0) v = 0.0;
                if (v > 255.0) v = 255.0;
                px[c] = (uint8_t)v;
            }
        }
    }
    free(sx); free(sy); free(base); free(amp); free(ct); free(st);
    free(bstart); free(bidx); free(bfill);
    return 0;
}

/* Region index map (nearest site, ties to the lowest index) by brute force:
 * used by tests to pin the bucketed search above. */
int synth_voronoi_sites_bruteforce(int32_t* out, int32_t w, int32_t h, int32_t regions,
                                   uint64_t seed) {
    if (!out || w < 1 || h < 1 || regions < 1) return 1;
    double* sx = (double*)malloc(sizeof(double) * regions);
    double* sy = (double*)malloc(sizeof(double) * regions);
    if (!sx || !sy) { free(sx); free(sy); return 2; }
    sm_stream site = {stream_key(seed, 1), 0};
    for (int i = 0; i < regions; i++) {
        sx[i] = u01(sm_next(&site)) * (double)w;
        sy[i] = u01(sm_next(&site)) * (double)h;
    }
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            double best = INFINITY;
            int bi = -1;
            for (int i = 0; i < regions; i++) {
                double dx = sx[i] - (double)x, dy = sy[i] - (double)y;
                double d2 = dx * dx + dy * dy;
                if (d2 < best) { best = d2; bi = i; }
            }
            out[(size_t)y * w + x] = bi;
        }
    free(sx); free(sy);
    return 0;
}
