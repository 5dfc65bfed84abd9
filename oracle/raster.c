/*
 * fp64 oracle: per-pixel front-to-back compositing and its exact derivative.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * HIP path is checked against. It shares no code with the HIP path and is
 * only built, loaded and called by tests/, the smoke check and the CPU
 * baseline leg of the benchmark.
 *
 * Method (3D Gaussian Splatting, the raster-based differentiable renderer the
 * paper instruments; the paper's Background section, "Differentiable
 * Rendering for Rasterization Pipelines", and the gradient-computation
 * outline of its Motivation section): every pixel walks the depth-ordered
 * list of Gaussians of its tile. For entry k with projected mean mu, conic
 * (A,B,C), opacity o and colour c:
 *     d     = p - mu,  p = (x + 0.5, y + 0.5)
 *     power = -0.5 (A dx^2 + C dy^2) - B dx dy
 *     skip the entry if power > 0
 *     alpha = min(0.99, o exp(power));  skip if alpha < 1/255
 *     stop (without compositing) if T (1 - alpha) < 1e-4
 *     I += alpha T c;  T *= (1 - alpha);  n_contrib = k (1-based position)
 * and finally I += T bg.  The backward pass returns, per Gaussian, the sum
 * over pixels of dL/d(mu_x, mu_y, A, B, C, o, c_r, c_g, c_b) for a given
 * dL/dI. That sum is what the paper's gradient kernel accumulates with
 * atomic adds, and what its warp-level reduction must reproduce (the reduced
 * result is the plain sum of the per-thread contributions).
 *
 * The derivative is written from the plain definition
 *     I = sum_k alpha_k T_k c_k + T_final bg,   T_k = prod_{j<k} (1 - alpha_j)
 * so dI/dalpha_k = T_k c_k - S_k / (1 - alpha_k) with S_k the colour behind
 * entry k (sum_{m>k} alpha_m T_m c_m + T_final bg). T_k is kept from the
 * forward product, never recovered by division.
 *
 * Every value is double. Decision margins are reported per pixel so a caller
 * can tell which pixels sit within rounding of a discrete decision.
 *
 * Threads (OpenMP, n_threads >= 1) only split independent work: the forward
 * takes image rows in parallel; the backward takes whole tiles, each adding
 * its pixels' contributions into one slot per tile-list entry, and the slots
 * are then added into the per-Gaussian sums in list order by one thread. The
 * result does not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_STOP 1e-4

typedef struct {
    int32_t width, height, tile, grid_x, grid_y;
    const int64_t *tile_start; /* [grid_x*grid_y + 1] offsets into ids */
    const int32_t *ids;        /* Gaussian index per list entry, depth order within a tile */
    const double *mean2d;      /* [n,2] */
    const double *conic;       /* [n,3] (A, B, C) */
    const double *opacity;     /* [n] */
    const double *rgb;         /* [n,3] */
    double bg[3];
    const uint8_t *tile_select; /* [grid_x*grid_y] or NULL = all tiles */
} oracle_frame;

typedef struct {
    int64_t pos;   /* 1-based position in the tile list */
    int32_t id;
    double alpha, T, G, power, dx, dy, clamped;
} entry;

static double rel(double a, double b) { return fabs(a - b) / fabs(b); }

/* Walk one pixel front to back; fills `out` with the composited entries.
 * Returns the number composited; writes colour, T_final, n_contrib, margin. */
static int64_t pixel_forward(const oracle_frame *f, int x, int y, entry *out,
                             double col[3], double *T_final, int32_t *n_contrib, double *margin,
                             uint64_t *sig)
{
    uint64_t h = 1469598103934665603ull; /* FNV-1a over (position, clamp state) of composited entries */
    int tile_id = (y / f->tile) * f->grid_x + (x / f->tile);
    int64_t beg = f->tile_start[tile_id], end = f->tile_start[tile_id + 1];
    double px = x + 0.5, py = y + 0.5;
    double T = 1.0;
    int64_t n = 0, last = 0;
    double m = INFINITY;
    col[0] = col[1] = col[2] = 0.0;
    for (int64_t k = beg; k < end; ++k) {
        int32_t g = f->ids[k];
        double dx = px - f->mean2d[2 * g + 0];
        double dy = py - f->mean2d[2 * g + 1];
        double A = f->conic[3 * g + 0], B = f->conic[3 * g + 1], C = f->conic[3 * g + 2];
        double qa = 0.5 * (A * dx * dx + C * dy * dy), qb = B * dx * dy;
        double power = -qa - qb;
        double scale = fabs(qa) + fabs(qb);
        if (scale > 0.0 && fabs(power) / scale < m) m = fabs(power) / scale;
        if (power > 0.0) continue;
        double G = exp(power);
        double raw = f->opacity[g] * G;
        double r1 = rel(raw, ALPHA_MIN), r2 = rel(raw, ALPHA_MAX);
        if (r1 < m) m = r1;
        if (r2 < m) m = r2;
        double alpha = raw < ALPHA_MAX ? raw : ALPHA_MAX;
        if (alpha < ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        double r3 = rel(Tn, T_STOP);
        if (r3 < m) m = r3;
        if (Tn < T_STOP) break;
        for (int c = 0; c < 3; ++c) col[c] += alpha * T * f->rgb[3 * g + c];
        {
            uint64_t word = (uint64_t)(k - beg + 1) * 2u + (raw > ALPHA_MAX ? 1u : 0u);
            for (int byte = 0; byte < 8; ++byte) { h ^= (word >> (8 * byte)) & 0xffu; h *= 1099511628211ull; }
        }
        if (out) {
            entry *e = &out[n];
            e->pos = k - beg + 1; e->id = g; e->alpha = alpha; e->T = T; e->G = G;
            e->power = power; e->dx = dx; e->dy = dy; e->clamped = raw > ALPHA_MAX;
        }
        n += 1;
        last = k - beg + 1;
        T = Tn;
    }
    for (int c = 0; c < 3; ++c) col[c] += T * f->bg[c];
    *T_final = T;
    *n_contrib = (int32_t)last;
    *margin = m;
    if (sig) *sig = h;
    return n;
}

static int selected(const oracle_frame *f, int x, int y)
{
    if (!f->tile_select) return 1;
    return f->tile_select[(y / f->tile) * f->grid_x + (x / f->tile)] != 0;
}

/* image [3,H,W], T_final [H,W], n_contrib [H,W], margin [H,W], sig [H,W]
 * (may be NULL): a hash of which entries were composited and whether their
 * alpha was clamped; n_used [H,W] (may be NULL): number of composited entries. Pixels of unselected tiles are left untouched. */
int oracle_render(const oracle_frame *f, double *image, double *T_final, int32_t *n_contrib, double *margin,
                  uint64_t *sig, int32_t *n_used, int n_threads)
{
    int64_t hw = (int64_t)f->width * f->height;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
    for (int y = 0; y < f->height; ++y)
        for (int x = 0; x < f->width; ++x) {
            if (!selected(f, x, y)) continue;
            int64_t p = (int64_t)y * f->width + x;
            double col[3];
            int64_t used = pixel_forward(f, x, y, NULL, col, &T_final[p], &n_contrib[p], &margin[p],
                                         sig ? &sig[p] : NULL);
            if (n_used) n_used[p] = (int32_t)used;
            for (int c = 0; c < 3; ++c) image[c * hw + p] = col[c];
        }
    return 0;
}

/* acc [n,9] += per-Gaussian sums of dL/d(mu_x, mu_y, A, B, C, o, r, g, b)
 * given dl_dimage [3,H,W]. `scratch_len` bounds the longest tile list. */
int oracle_backward(const oracle_frame *f, const double *dl_dimage, double *acc, int64_t scratch_len,
                    int n_threads)
{
    int64_t hw = (int64_t)f->width * f->height;
    int ntiles = f->grid_x * f->grid_y;
    int64_t P = f->tile_start[ntiles];
    /* slot[9 k + j]: value j summed over the pixels of the tile that list entry k belongs to */
    double *slot = (double *)calloc((size_t)(P > 0 ? P : 1) * 9, sizeof(double));
    if (!slot) return -1;
    int failed = 0;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        entry *ent = (entry *)malloc(sizeof(entry) * (size_t)(scratch_len > 0 ? scratch_len : 1));
        if (!ent) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int t = 0; t < ntiles; ++t) {
            if (!ent) continue;
            if (f->tile_select && !f->tile_select[t]) continue;
            int64_t beg = f->tile_start[t];
            int tx = t % f->grid_x, ty = t / f->grid_x;
            int y1 = (ty + 1) * f->tile < f->height ? (ty + 1) * f->tile : f->height;
            int x1 = (tx + 1) * f->tile < f->width ? (tx + 1) * f->tile : f->width;
            for (int y = ty * f->tile; y < y1; ++y)
                for (int x = tx * f->tile; x < x1; ++x) {
                    int64_t p = (int64_t)y * f->width + x;
                    double col[3], Tf, mg;
                    int32_t nc;
                    int64_t n = pixel_forward(f, x, y, ent, col, &Tf, &nc, &mg, NULL);
                    double G[3] = {dl_dimage[p], dl_dimage[hw + p], dl_dimage[2 * hw + p]};
                    /* S = colour behind the current entry, starting with the background. */
                    double S[3] = {Tf * f->bg[0], Tf * f->bg[1], Tf * f->bg[2]};
                    for (int64_t i = n - 1; i >= 0; --i) {
                        const entry *e = &ent[i];
                        const double *c = &f->rgb[3 * e->id];
                        double *a = &slot[9 * (beg + e->pos - 1)];
                        double dL_dalpha = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            a[6 + ch] += e->alpha * e->T * G[ch];
                            dL_dalpha += (e->T * c[ch] - S[ch] / (1.0 - e->alpha)) * G[ch];
                        }
                        for (int ch = 0; ch < 3; ++ch) S[ch] += e->alpha * e->T * c[ch];
                        /* alpha = min(0.99, o G): no dependence on o or power when clamped. */
                        if (e->clamped) continue;
                        double o = f->opacity[e->id];
                        a[5] += dL_dalpha * e->G;                 /* dalpha/do = G */
                        double dL_dpower = dL_dalpha * o * e->G;  /* dalpha/dpower = o G */
                        const double *K = &f->conic[3 * e->id];
                        /* d = p - mu, so dpower/dmu = (A dx + B dy, B dx + C dy). */
                        a[0] += dL_dpower * (K[0] * e->dx + K[1] * e->dy);
                        a[1] += dL_dpower * (K[1] * e->dx + K[2] * e->dy);
                        a[2] += dL_dpower * (-0.5 * e->dx * e->dx);
                        a[3] += dL_dpower * (-e->dx * e->dy);
                        a[4] += dL_dpower * (-0.5 * e->dy * e->dy);
                    }
                }
        }
        free(ent);
    }
    if (!failed)
        for (int64_t k = 0; k < P; ++k) {
            double *a = &acc[9 * (int64_t)f->ids[k]];
            for (int j = 0; j < 9; ++j) a[j] += slot[9 * k + j];
        }
    free(slot);
    return failed ? -1 : 0;
}

/* Per-pixel list of composited entries (positions and Gaussian ids), for
 * tests that compare decisions; returns the count written (<= cap). */
int64_t oracle_pixel_entries(const oracle_frame *f, int x, int y, int64_t *pos, int32_t *ids, int64_t cap)
{
    int tile_id = (y / f->tile) * f->grid_x + (x / f->tile);
    int64_t len = f->tile_start[tile_id + 1] - f->tile_start[tile_id];
    entry *ent = (entry *)malloc(sizeof(entry) * (size_t)(len > 0 ? len : 1));
    if (!ent) return -1;
    double col[3], Tf, mg;
    int32_t nc;
    int64_t n = pixel_forward(f, x, y, ent, col, &Tf, &nc, &mg, NULL);
    int64_t w = n < cap ? n : cap;
    for (int64_t i = 0; i < w; ++i) { pos[i] = ent[i].pos; ids[i] = ent[i].id; }
    free(ent);
    return n;
}
