/*
 * Seeded synthetic graph generators (edge lists only).
 *
 * This file holds no part of the triangle-counting method: it only draws
 * vertex pairs. Both the CPU oracle and the GPU library are fed the arrays
 * it writes, so the two sides always see identical inputs.
 *
 * Every random number is a pure function of (seed, stream, counter): a
 * SplitMix64 finaliser applied to a Weyl sequence (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014). Outputs
 * therefore do not depend on the OpenMP thread count or schedule.
 *
 * Output layout everywhere: int32 pairs, row-major [E][2].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* One 64-bit draw for (seed, stream, ctr). */
static inline uint64_t draw64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t key = mix64(seed * GOLDEN + stream * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull);
    return mix64(key + (ctr + 1) * GOLDEN);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double draw_unit(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return (double)(draw64(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, bound) by Lemire's multiply-shift (bias < bound/2^64). */
static inline uint64_t draw_below(uint64_t seed, uint64_t stream, uint64_t ctr, uint64_t bound) {
    return (uint64_t)(((__uint128_t)draw64(seed, stream, ctr) * bound) >> 64);
}

enum { ST_RMAT = 1, ST_PERM = 2, ST_FLIP = 3, ST_CL = 4, ST_RGG = 5, ST_SHUF = 6 };

/* Fisher-Yates permutation of [0, n) (sequential; n up to 2^31). */
void gg_permutation(int32_t n, uint64_t seed, int32_t* perm) {
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = (int64_t)n - 1; i > 0; --i) {
        int64_t j = (int64_t)draw_below(seed, ST_PERM, (uint64_t)i, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each of the E draws picks
 * one quadrant per bit level with probabilities a, b, c, d = 1-a-b-c; the
 * row bit is 1 for quadrants c, d and the column bit is 1 for b, d. No noise.
 * If perm is non-NULL both endpoints are mapped through it. With flip != 0
 * each pair is written in a random direction.
 */
void gg_rmat(int32_t scale, int64_t E, double a, double b, double c, uint64_t seed,
             const int32_t* perm, int32_t flip, int32_t* out) {
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E; ++i) {
        uint32_t u = 0, v = 0;
        for (int32_t l = 0; l < scale; ++l) {
            double r = draw_unit(seed, ST_RMAT, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
            uint32_t bu = (r >= ab) ? 1u : 0u;
            uint32_t bv = ((r >= a && r < ab) || r >= abc) ? 1u : 0u;
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        int32_t x = perm ? perm[u] : (int32_t)u;
        int32_t y = perm ? perm[v] : (int32_t)v;
        if (flip && (draw64(seed, ST_FLIP, (uint64_t)i) & 1ull)) { int32_t t = x; x = y; y = t; }
        out[2 * i] = x;
        out[2 * i + 1] = y;
    }
}

/*
 * Chung-Lu (Chung and Lu, PNAS 2002) with E independent endpoint pairs, each
 * endpoint drawn with probability proportional to w_i = (i+1)^(-1/(gamma-1))
 * by inverse-CDF search over the cumulative weights. Ids are then mapped
 * through perm (if non-NULL) and offset by base.
 */
void gg_chung_lu(int32_t n, int64_t E, double gamma, uint64_t seed, const int32_t* perm,
                 int32_t base, int32_t* out) {
    double* cdf = (double*)malloc(sizeof(double) * (size_t)n);
    double acc = 0.0, ex = -1.0 / (gamma - 1.0);
    for (int32_t i = 0; i < n; ++i) { acc += pow((double)i + 1.0, ex); cdf[i] = acc; }
#pragma omp parallel for schedule(static) if (E > 65536)
    for (int64_t i = 0; i < 2 * E; ++i) {
        double r = draw_unit(seed, ST_CL, (uint64_t)i) * acc;
        int32_t lo = 0, hi = n - 1;            /* first index with cdf > r */
        while (lo < hi) {
            int32_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > r) hi = mid; else lo = mid + 1;
        }
        out[i] = base + (perm ? perm[lo] : lo);
    }
    free(cdf);
}

/*
 * Random geometric graph: n points uniform in [0,1)^2 (x = draw 2i, y =
 * draw 2i+1), an edge for every pair at Euclidean distance <= r (compared as
 * squared distances in double). Pairs are found through a grid of cells of
 * side >= r. Writes at most cap pairs (i < j) and returns the total number of
 * pairs, so a caller whose cap was too small can retry.
 */
int64_t gg_rgg(int32_t n, double r, uint64_t seed, int32_t* out, int64_t cap) {
    int32_t g = (int32_t)floor(1.0 / r);
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    int64_t ncell = (int64_t)g * g;
    double* xy = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    int64_t* cstart = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* per_pt = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        xy[2 * i] = draw_unit(seed, ST_RGG, 2 * (uint64_t)i);
        xy[2 * i + 1] = draw_unit(seed, ST_RGG, 2 * (uint64_t)i + 1);
        int32_t cx = (int32_t)(xy[2 * i] * g), cy = (int32_t)(xy[2 * i + 1] * g);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        cell_of[i] = cy * g + cx;
    }
    for (int64_t i = 0; i < n; ++i) cstart[cell_of[i] + 1]++;
    for (int64_t k = 0; k < ncell; ++k) cstart[k + 1] += cstart[k];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
        memcpy(fill, cstart, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = (int32_t)i;
        free(fill);
    }
    const double r2 = r * r;
    /* pass 1: pairs per point (each pair counted at its smaller id) */
    for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i) {
            int32_t c = cell_of[i], cx = c % g, cy = c / g;
            int64_t cnt = 0, w = pass ? per_pt[i] : 0;
            for (int32_t dy = -1; dy <= 1; ++dy) {
                int32_t yy = cy + dy;
                if (yy < 0 || yy >= g) continue;
                for (int32_t dx = -1; dx <= 1; ++dx) {
                    int32_t xx = cx + dx;
                    if (xx < 0 || xx >= g) continue;
                    int64_t k = (int64_t)yy * g + xx;
                    for (int64_t p = cstart[k]; p < cstart[k + 1]; ++p) {
                        int32_t j = order[p];
                        if (j <= i) continue;
                        double ddx = xy[2 * i] - xy[2 * (int64_t)j];
                        double ddy = xy[2 * i + 1] - xy[2 * (int64_t)j + 1];
                        if (ddx * ddx + ddy * ddy <= r2) {
                            if (pass && w < cap) { out[2 * w] = (int32_t)i; out[2 * w + 1] = j; }
                            ++w; ++cnt;
                        }
                    }
                }
            }
            if (!pass) per_pt[i] = cnt;
        }
        if (!pass) {   /* exclusive scan of per-point counts */
            int64_t run = 0;
            for (int64_t i = 0; i < n; ++i) { int64_t t = per_pt[i]; per_pt[i] = run; run += t; }
            per_pt[n] = run;
        }
    }
    int64_t total = per_pt[n];
    free(xy); free(cstart); free(cell_of); free(order); free(per_pt);
    return total;
}

/*
 * Random order and direction for an edge list, in place: a Fisher-Yates
 * shuffle of the pairs followed by a random flip of each pair.
 */
void gg_shuffle_edges(int32_t* e, int64_t E, uint64_t seed) {
    for (int64_t i = E - 1; i > 0; --i) {
        int64_t j = (int64_t)draw_below(seed, ST_SHUF, (uint64_t)i, (uint64_t)i + 1);
        int32_t a = e[2 * i], b = e[2 * i + 1];
        e[2 * i] = e[2 * j]; e[2 * i + 1] = e[2 * j + 1];
        e[2 * j] = a; e[2 * j + 1] = b;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < E; ++i) {
        if (draw64(seed, ST_FLIP, (uint64_t)i) & 1ull) {
            int32_t a = e[2 * i]; e[2 * i] = e[2 * i + 1]; e[2 * i + 1] = a;
        }
    }
}

/* Raw 64-bit draws (exposed so tests can check the generator's statistics). */
void gg_draws(uint64_t seed, uint64_t stream, int64_t count, uint64_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = draw64(seed, stream, (uint64_t)i);
}
