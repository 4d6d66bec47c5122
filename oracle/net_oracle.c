/*
 * CPU oracle for the learned warm start: a small convolutional net that
 * predicts, for every pixel, which of the nine grid cells around it (the
 * candidate set of Section 3's association) holds the centre it converges
 * to, so that a few iterations from that labelling replace many from the
 * plain grid seeds (Section 1: fewer iterations are faster but worse).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; it shares no code with the GPU
 * library.
 *
 * Net: x = (L/100, a/128, b/128); conv 3x3 3->32, ReLU; conv 3x3 32->32,
 * ReLU; conv 3x3 32->9; logits = conv output + P[phase], phase =
 * (y mod S)*S + (x mod S) in full-image coordinates (a learned per-phase
 * bias: the convolutions are translation-equivariant and cannot see where a
 * pixel lies inside its cell).  Zero padding outside the evaluated region at
 * every layer.  Weights W[tap][out][in], tap = (dy+1)*3 + (dx+1) reading the
 * input at (x+dx, y+dy).
 *
 * Threads: the convolutions' output rows are split over OpenMP threads when
 * built with -fopenmp (each output is the same sum in the same order);
 * gradient sums over pixels stay sequential.
 *
 * Arithmetic: FP64 throughout.  With bf16 != 0 the values the GPU stores in
 * bfloat16 are rounded to bfloat16 (round to nearest even) at the same
 * points: the input x, the convolution weights, the ReLU outputs a1 and a2.
 * Biases, P and the logits stay unrounded.  With bf16 == 0 the net is plain
 * FP64 (for finite-difference checks of the backward pass).
 *
 * Loss: mean over pixels of the softmax cross-entropy against the target
 * class (pixels with target < 0 are ignored).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define C1 32
#define C2 32
#define C3 9

enum { OFF_W1 = 0, OFF_B1 = 9 * C1 * 3, OFF_W2 = OFF_B1 + C1, OFF_B2 = OFF_W2 + 9 * C2 * C1,
       OFF_W3 = OFF_B2 + C2, OFF_B3 = OFF_W3 + 9 * C3 * C2, OFF_P = OFF_B3 + C3 };

int orn_param_count(int S) { return OFF_P + S * S * C3; }

/* bfloat16 round to nearest even of a float, returned as double */
static double bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

double orn_bf16(double v) { return bf16(v); }

static double rnd(int on, double v) { return on ? bf16(v) : v; }

typedef struct {
    int w, h, ox, oy, S, bf;
    const double* p;
    double* W1r; /* rounded copies of the convolution weights */
    double* W2r;
    double* W3r;
    double* x;  /* [h][w][3] */
    double* a1; /* [h][w][C1] */
    double* a2; /* [h][w][C2] */
    double* lg; /* [h][w][C3] */
} net_t;

static void conv(const net_t* n, const double* in, int cin, const double* W, const double* b,
                 int cout, int relu, int round_out, double* out) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < n->h; y++)
        for (int x = 0; x < n->w; x++) {
            double* o = out + ((size_t)y * n->w + x) * cout;
            for (int co = 0; co < cout; co++) {
                double s = b[co];
                for (int t = 0; t < 9; t++) {
                    int xx = x + t % 3 - 1, yy = y + t / 3 - 1;
                    if (xx < 0 || yy < 0 || xx >= n->w || yy >= n->h) continue;
                    const double* v = in + ((size_t)yy * n->w + xx) * cin;
                    const double* wr = W + ((size_t)t * cout + co) * cin;
                    for (int ci = 0; ci < cin; ci++) s += wr[ci] * v[ci];
                }
                if (relu && s < 0.0) s = 0.0;
                o[co] = round_out ? rnd(n->bf, s) : s;
            }
        }
}

static int net_forward(net_t* n) {
    size_t np = (size_t)n->w * n->h;
    n->W1r = malloc(sizeof(double) * 9 * C1 * 3);
    n->W2r = malloc(sizeof(double) * 9 * C2 * C1);
    n->W3r = malloc(sizeof(double) * 9 * C3 * C2);
    n->a1 = malloc(sizeof(double) * np * C1);
    n->a2 = malloc(sizeof(double) * np * C2);
    if (!n->W1r || !n->W2r || !n->W3r || !n->a1 || !n->a2) return 2;
    for (int i = 0; i < 9 * C1 * 3; i++) n->W1r[i] = rnd(n->bf, n->p[OFF_W1 + i]);
    for (int i = 0; i < 9 * C2 * C1; i++) n->W2r[i] = rnd(n->bf, n->p[OFF_W2 + i]);
    for (int i = 0; i < 9 * C3 * C2; i++) n->W3r[i] = rnd(n->bf, n->p[OFF_W3 + i]);
    conv(n, n->x, 3, n->W1r, n->p + OFF_B1, C1, 1, 1, n->a1);
    conv(n, n->a1, C1, n->W2r, n->p + OFF_B2, C2, 1, 1, n->a2);
    conv(n, n->a2, C2, n->W3r, n->p + OFF_B3, C3, 0, 0, n->lg);
    for (int y = 0; y < n->h; y++)
        for (int x = 0; x < n->w; x++) {
            int ph = ((y + n->oy) % n->S) * n->S + (x + n->ox) % n->S;
            for (int c = 0; c < C3; c++) n->lg[((size_t)y * n->w + x) * C3 + c] += n->p[OFF_P + ph * C3 + c];
        }
    return 0;
}

static void net_free(net_t* n) {
    free(n->W1r); free(n->W2r); free(n->W3r); free(n->a1); free(n->a2); free(n->x);
}

static int net_init(net_t* n, int w, int h, int ox, int oy, int S, const float* L, const float* A,
                    const float* B, const double* params, int bf) {
    memset(n, 0, sizeof(*n));
    if (w < 1 || h < 1 || S < 1 || ox < 0 || oy < 0 || !L || !A || !B || !params) return 1;
    n->w = w; n->h = h; n->ox = ox; n->oy = oy; n->S = S; n->bf = bf; n->p = params;
    size_t np = (size_t)w * h;
    n->x = malloc(sizeof(double) * np * 3);
    if (!n->x) return 2;
    for (size_t i = 0; i < np; i++) {
        n->x[3 * i + 0] = rnd(bf, (double)(L[i] / 100.0f));
        n->x[3 * i + 1] = rnd(bf, (double)(A[i] / 128.0f));
        n->x[3 * i + 2] = rnd(bf, (double)(B[i] / 128.0f));
    }
    return 0;
}

/* logits[h][w][9]; a1/a2 (may be NULL) receive the ReLU outputs */
int orn_forward(int w, int h, int ox, int oy, int S, const float* L, const float* A, const float* B,
                const double* params, int bf, double* logits, double* a1, double* a2) {
    net_t n;
    int rc = net_init(&n, w, h, ox, oy, S, L, A, B, params, bf);
    if (rc) { net_free(&n); return rc; }
    if (!logits) { net_free(&n); return 1; }
    n.lg = logits;
    rc = net_forward(&n);
    if (!rc) {
        size_t np = (size_t)w * h;
        if (a1) memcpy(a1, n.a1, sizeof(double) * np * C1);
        if (a2) memcpy(a2, n.a2, sizeof(double) * np * C2);
    }
    net_free(&n);
    return rc;
}

/* Mean softmax cross-entropy and (grad != NULL) its gradient with respect
 * to every parameter (for the convolution weights: with respect to the
 * rounded weights, passed straight through to the FP32 masters). */
int orn_loss_grad(int w, int h, int ox, int oy, int S, const float* L, const float* A, const float* B,
                  const int32_t* target, const double* params, int bf, double* loss, double* grad) {
    net_t n;
    int rc = net_init(&n, w, h, ox, oy, S, L, A, B, params, bf);
    size_t np = (size_t)w * h;
    double* lg = malloc(sizeof(double) * np * C3);
    double* d3 = malloc(sizeof(double) * np * C3);
    double* d2 = malloc(sizeof(double) * np * C2);
    double* d1 = malloc(sizeof(double) * np * C1);
    if (rc || !lg || !d3 || !d2 || !d1 || !target || !loss) {
        net_free(&n); free(lg); free(d3); free(d2); free(d1);
        return rc ? rc : 1;
    }
    n.lg = lg;
    rc = net_forward(&n);
    if (rc) { net_free(&n); free(lg); free(d3); free(d2); free(d1); return rc; }
    size_t counted = 0;
    for (size_t i = 0; i < np; i++) counted += target[i] >= 0;
    double total = 0.0;
    for (size_t i = 0; i < np; i++) {
        const double* l = lg + i * C3;
        double* d = d3 + i * C3;
        if (target[i] < 0 || target[i] >= C3) {
            for (int c = 0; c < C3; c++) d[c] = 0.0;
            continue;
        }
        double m = l[0];
        for (int c = 1; c < C3; c++) if (l[c] > m) m = l[c];
        double se = 0.0;
        for (int c = 0; c < C3; c++) se += exp(l[c] - m);
        total += (m + log(se)) - l[target[i]];
        for (int c = 0; c < C3; c++) {
            double pr = exp(l[c] - m) / se;
            d[c] = (pr - (c == target[i] ? 1.0 : 0.0)) / (double)(counted ? counted : 1);
        }
    }
    *loss = counted ? total / (double)counted : 0.0;
    if (!grad) { net_free(&n); free(lg); free(d3); free(d2); free(d1); return 0; }
    memset(grad, 0, sizeof(double) * orn_param_count(S));
    /* per-phase bias and conv3 */
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int ph = ((y + oy) % S) * S + (x + ox) % S;
            const double* d = d3 + ((size_t)y * w + x) * C3;
            for (int c = 0; c < C3; c++) {
                grad[OFF_P + ph * C3 + c] += d[c];
                grad[OFF_B3 + c] += d[c];
            }
        }
    /* backward of one convolution: dout [np][cout] -> dW, db (given), din */
#define CONV_BACK(IN, CIN, WR, OFFW, DOUT, COUT, DIN)                                            \
    do {                                                                                         \
        if (DIN) memset(DIN, 0, sizeof(double) * np * (CIN));                                    \
        for (int y = 0; y < h; y++)                                                              \
            for (int x = 0; x < w; x++) {                                                        \
                const double* dout = (DOUT) + ((size_t)y * w + x) * (COUT);                      \
                for (int t = 0; t < 9; t++) {                                                    \
                    int xx = x + t % 3 - 1, yy = y + t / 3 - 1;                                  \
                    if (xx < 0 || yy < 0 || xx >= w || yy >= h) continue;                        \
                    const double* v = (IN) + ((size_t)yy * w + xx) * (CIN);                      \
                    double* dv = (DIN) ? (DIN) + ((size_t)yy * w + xx) * (CIN) : NULL;           \
                    for (int co = 0; co < (COUT); co++) {                                        \
                        const double g = dout[co];                                               \
                        double* gw = grad + (OFFW) + ((size_t)t * (COUT) + co) * (CIN);          \
                        const double* wr = (WR) + ((size_t)t * (COUT) + co) * (CIN);             \
                        for (int ci = 0; ci < (CIN); ci++) {                                     \
                            gw[ci] += g * v[ci];                                                 \
                            if (dv) dv[ci] += g * wr[ci];                                        \
                        }                                                                        \
                    }                                                                            \
                }                                                                                \
            }                                                                                    \
    } while (0)
    CONV_BACK(n.a2, C2, n.W3r, OFF_W3, d3, C3, d2);
    for (size_t i = 0; i < np * C2; i++) if (!(n.a2[i] > 0.0)) d2[i] = 0.0;  /* ReLU */
    for (size_t i = 0; i < np; i++)
        for (int c = 0; c < C2; c++) grad[OFF_B2 + c] += d2[i * C2 + c];
    CONV_BACK(n.a1, C1, n.W2r, OFF_W2, d2, C2, d1);
    for (size_t i = 0; i < np * C1; i++) if (!(n.a1[i] > 0.0)) d1[i] = 0.0;
    for (size_t i = 0; i < np; i++)
        for (int c = 0; c < C1; c++) grad[OFF_B1 + c] += d1[i * C1 + c];
    double* none = NULL;
    CONV_BACK(n.x, 3, n.W1r, OFF_W1, d1, C1, none);
#undef CONV_BACK
    net_free(&n); free(lg); free(d3); free(d2); free(d1);
    return 0;
}

/* Warm-start labels: the argmax class (ties to the lowest class) names the
 * cell (gy + c/3 - 1, gx + c%3 - 1) around the pixel's own cell, clamped
 * into the ns_c x ns_r grid. */
int orn_decode(int w, int h, int S, const double* logits, int32_t* labels) {
    if (w < 1 || h < 1 || S < 1 || !logits || !labels) return 1;
    int ns_c = (w + S - 1) / S, ns_r = (h + S - 1) / S;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            const double* l = logits + ((size_t)y * w + x) * C3;
            int best = 0;
            for (int c = 1; c < C3; c++) if (l[c] > l[best]) best = c;
            int cy = y / S + best / 3 - 1, cx = x / S + best % 3 - 1;
            if (cy < 0) cy = 0;
            if (cy >= ns_r) cy = ns_r - 1;
            if (cx < 0) cx = 0;
            if (cx >= ns_c) cx = ns_c - 1;
            labels[(size_t)y * w + x] = cy * ns_c + cx;
        }
    return 0;
}

/* Which decoded pixels vote in the first centre update: those whose best
 * class has softmax probability at least tau, i.e. sum_c exp(l_c - l_best)
 * * tau <= 1 (FP64).  tau = 0: every pixel; tau > 1: none.  The others keep
 * their decoded label but leave the first update to the confident pixels,
 * whose colours are purer (a reading of the extension's decode, not a step
 * of the paper). */
int orn_votes(int w, int h, const double* logits, double tau, uint8_t* votes) {
    if (w < 1 || h < 1 || !logits || !votes || !(tau >= 0.0)) return 1;
    for (size_t i = 0; i < (size_t)w * h; i++) {
        const double* l = logits + i * C3;
        int best = 0;
        for (int c = 1; c < C3; c++) if (l[c] > l[best]) best = c;
        double s = 0.0;
        for (int c = 0; c < C3; c++) s += exp(l[c] - l[best]);
        votes[i] = s * tau <= 1.0;
    }
    return 0;
}

/* Training target: the class of the cell holding the pixel's label relative
 * to the pixel's own cell, (dy+1)*3 + (dx+1); -1 if it is not a neighbour. */
int orn_targets(int w, int h, int S, const int32_t* labels, int32_t* target) {
    if (w < 1 || h < 1 || S < 1 || !labels || !target) return 1;
    int ns_c = (w + S - 1) / S;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int k = labels[(size_t)y * w + x];
            int dy = k / ns_c - y / S, dx = k % ns_c - x / S;
            target[(size_t)y * w + x] =
                (dx < -1 || dx > 1 || dy < -1 || dy > 1) ? -1 : (dy + 1) * 3 + (dx + 1);
        }
    return 0;
}
