/*
 * CPU oracle for exhaustive range-domain matching (test infrastructure only).
 *
 * This file is part of the test oracle. Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg load it; the GPU library never does,
 * and the two share no code.
 *
 * It is deliberately plain and slow. For every range block R and every
 * candidate (domain j, isometry t, contrast index) it evaluates the distance of
 * eq. (1), E = sum_i (s*d_i + o - r_i)^2, with the offset o of eq. (3),
 * o = mean(R) - s*mean(D), literally pixel by pixel (Section 2). Nothing is
 * blocked, fused or reordered.
 *
 * Exactness. The decimated domain d is the 2x2 mean, d_i = dd_i / 4, where
 * dd_i is an integer sum of four pixels. The contrast is s = k / 10 (Q = 10).
 * Multiplying each residual by 4*Q*n makes it an integer:
 *     e_i = k*n*dd_i + 4*Q*sumR - k*sumDD - 4*Q*n*r_i,
 * so E = (sum_i e_i^2) / (4*Q*n)^2 and sum_i e_i^2 is exact in int64
 * (|e_i| < 2^23 and n <= 256). The argmin is taken on these exact integers.
 * Ties go to the lexicographically smallest (E, j, t, s_idx).
 *
 * Isometries (Section 2: the identity, clockwise rotations by 90, 180 and
 * 270 degrees, and the mirror images of those four). On a B x B block with
 * row i and column c:
 *   t=0  out[i][c] = in[i][c]
 *   t=1  out[i][c] = in[B-1-c][i]          (90 degrees clockwise)
 *   t=2  out[i][c] = in[B-1-i][B-1-c]      (180 degrees)
 *   t=3  out[i][c] = in[c][B-1-i]          (270 degrees clockwise)
 *   t=4+u  out[i][c] = rot_u(in)[i][B-1-c] (left-right mirror of t=u)
 * The candidate compared with R is T_t applied to the decimated domain.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_Q 10

/* Index into a B x B input block of the pixel that T_t places at (i, c). */
static int iso_src(int B, int t, int i, int c)
{
    if (t >= 4) {
        c = B - 1 - c;
        t -= 4;
    }
    switch (t) {
    case 0: return i * B + c;
    case 1: return (B - 1 - c) * B + i;
    case 2: return (B - 1 - i) * B + (B - 1 - c);
    default: return c * B + (B - 1 - i);
    }
}

/* Decimated domain (4x the 2x2 mean) of the 2B x 2B block at (y, x). */
static void decimate(const uint8_t *img, int pitch, int y, int x, int B, int64_t *dd)
{
    for (int i = 0; i < B; ++i)
        for (int c = 0; c < B; ++c) {
            const uint8_t *p = img + (int64_t)(y + 2 * i) * pitch + (x + 2 * c);
            dd[i * B + c] = (int64_t)p[0] + p[1] + p[pitch] + p[pitch + 1];
        }
}

/* sum_i e_i^2 of eq. (1) for one candidate, times (4 Q n)^2. */
static int64_t literal_e(const int64_t *r, const int64_t *cand, int n, int k)
{
    int64_t sr = 0, sd = 0;
    for (int i = 0; i < n; ++i) {
        sr += r[i];
        sd += cand[i];
    }
    int64_t e2 = 0;
    for (int i = 0; i < n; ++i) {
        int64_t e = (int64_t)k * n * cand[i] + 4 * ORC_Q * sr - (int64_t)k * sd
                  - (int64_t)4 * ORC_Q * n * r[i];
        e2 += e * e;
    }
    return e2;
}

typedef struct {
    int64_t e;
    int32_t j, t, s;
} cand_t;

static int cand_less(const cand_t *a, const cand_t *b)
{
    if (a->e != b->e) return a->e < b->e;
    if (a->j != b->j) return a->j < b->j;
    if (a->t != b->t) return a->t < b->t;
    return a->s < b->s;
}

/* One candidate: E * (4 Q n)^2 for range block r (B x B, values 0..255) and
 * decimated domain dd (B x B, values 0..1020) under isometry t and s = k/10. */
int64_t orc_eval(const int32_t *r, const int32_t *dd, int B, int t, int k)
{
    int n = B * B;
    int64_t *rv = malloc(sizeof(int64_t) * n);
    int64_t *dv = malloc(sizeof(int64_t) * n);
    int64_t *cv = malloc(sizeof(int64_t) * n);
    for (int i = 0; i < n; ++i) {
        rv[i] = r[i];
        dv[i] = dd[i];
    }
    for (int i = 0; i < B; ++i)
        for (int c = 0; c < B; ++c)
            cv[i * B + c] = dv[iso_src(B, t, i, c)];
    int64_t e = literal_e(rv, cv, n, k);
    free(rv);
    free(dv);
    free(cv);
    return e;
}

/* Apply isometry t to a B x B int32 block (used by tests to pin the table). */
void orc_isometry(const int32_t *in, int B, int t, int32_t *out)
{
    for (int i = 0; i < B; ++i)
        for (int c = 0; c < B; ++c)
            out[i * B + c] = in[iso_src(B, t, i, c)];
}

/*
 * Exhaustive search at one level.
 *   img, H, W, pitch : uint8 image, row-major
 *   B, L             : range side and domain step
 *   s_k, n_s         : contrast numerators (s = k/10), searched in this order
 *   pool, n_pool     : domain indices on the unfiltered grid (row-major over
 *                      top-left corners y = L*dy, x = L*dx, 0 <= y,x <= H,W - 2B)
 *   ranges_yx, n_r   : top-left corners of the range blocks (pairs y, x)
 * Outputs per range: best E*(4Qn)^2, domain, isometry, contrast index, and the
 * second-smallest E*(4Qn)^2 over all other candidates (equal to the best on a
 * tie). Returns 0, or -1 on an argument error.
 */
int orc_match_level(const uint8_t *img, int H, int W, int pitch, int B, int L,
                    const int32_t *s_k, int n_s, const int32_t *pool, int n_pool,
                    const int32_t *ranges_yx, int n_r, int64_t *best_e, int32_t *best_j,
                    int32_t *best_t, int32_t *best_s, int64_t *second_e)
{
    if (B < 1 || L < 1 || 2 * B > H || 2 * B > W || n_pool < 1 || n_s < 1) return -1;
    int gx = (W - 2 * B) / L + 1;
    int n = B * B;
#pragma omp parallel
    {
        int64_t *r = malloc(sizeof(int64_t) * n);
        int64_t *dd = malloc(sizeof(int64_t) * n);
        int64_t *cand = malloc(sizeof(int64_t) * n);
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < n_r; ++q) {
            int ry = ranges_yx[2 * q], rx = ranges_yx[2 * q + 1];
            for (int i = 0; i < B; ++i)
                for (int c = 0; c < B; ++c)
                    r[i * B + c] = img[(int64_t)(ry + i) * pitch + rx + c];
            cand_t best = {INT64_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
            cand_t second = best;
            for (int p = 0; p < n_pool; ++p) {
                int j = pool[p];
                int y = (j / gx) * L, x = (j % gx) * L;
                decimate(img, pitch, y, x, B, dd);
                for (int t = 0; t < 8; ++t) {
                    for (int i = 0; i < B; ++i)
                        for (int c = 0; c < B; ++c)
                            cand[i * B + c] = dd[iso_src(B, t, i, c)];
                    for (int s = 0; s < n_s; ++s) {
                        cand_t cur = {literal_e(r, cand, n, s_k[s]), j, t, s};
                        if (cand_less(&cur, &best)) {
                            second = best;
                            best = cur;
                        } else if (cand_less(&cur, &second)) {
                            second = cur;
                        }
                    }
                }
            }
            best_e[q] = best.e;
            best_j[q] = best.j;
            best_t[q] = best.t;
            best_s[q] = best.s;
            second_e[q] = second.e;
        }
        free(r);
        free(dd);
        free(cand);
    }
    return 0;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
