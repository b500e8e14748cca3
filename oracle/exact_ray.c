/*
 * exact_ray.c -- exact line integrals through a piecewise-constant voxel grid.
 *
 * TEST INFRASTRUCTURE ONLY (a brute-force reference used to pin the oracle; see
 * ctoracle.c).  It shares no code with ctoracle.c or with the HIP engine: it does not know
 * about footprints, detectors or gantry poses, only about segments and boxes.
 *
 * For a segment a -> b the integral is the sum over voxels of (length of the segment inside
 * the voxel) x (voxel value).  The segment is cut at every crossing with a grid plane
 * (parametric crossings, as in Siddon's method); each piece lies in one voxel, found from the
 * piece's midpoint.  Double precision throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static int cmp_double(const void *pa, const void *pb)
{
    const double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

/* Grid: n[3] voxels with pitch h[3]; voxel (ix, iy, iz) occupies
 * [o_k + (i_k - n_k/2) h_k, o_k + (i_k + 1 - n_k/2) h_k] along each axis k.
 * vol is [n2][n1][n0] (axis 0 fastest). */
static double one_ray(const double *vol, const int n[3], const double h[3], const double o[3],
                      const double a[3], const double b[3], double *alpha)
{
    double dir[3];
    for (int k = 0; k < 3; ++k)
        dir[k] = b[k] - a[k];
    const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    int m = 0;
    alpha[m++] = 0.0;
    alpha[m++] = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (dir[k] == 0.0)
            continue;
        for (int p = 0; p <= n[k]; ++p) {
            const double plane = o[k] + (p - 0.5 * n[k]) * h[k];
            const double t = (plane - a[k]) / dir[k];
            if (t > 0.0 && t < 1.0)
                alpha[m++] = t;
        }
    }
    qsort(alpha, (size_t)m, sizeof(double), cmp_double);
    double acc = 0.0;
    for (int q = 0; q + 1 < m; ++q) {
        const double t0 = alpha[q], t1 = alpha[q + 1];
        if (t1 <= t0)
            continue;
        const double tm = 0.5 * (t0 + t1);
        int idx[3], inside = 1;
        for (int k = 0; k < 3; ++k) {
            const double c = a[k] + tm * dir[k];
            const double f = floor((c - o[k]) / h[k] + 0.5 * n[k]);
            if (f < 0.0 || f >= n[k]) {
                inside = 0;
                break;
            }
            idx[k] = (int)f;
        }
        if (!inside)
            continue;
        const double val = vol[((int64_t)idx[2] * n[1] + idx[1]) * n[0] + idx[0]];
        acc += (t1 - t0) * len * val;
    }
    return acc;
}

/* out[r] = integral of the grid along segment a[r] -> b[r] (a, b: [n_rays][3]). */
int exr_integrals(const double *vol, const int32_t *n, const double *h, const double *o,
                  int64_t n_rays, const double *a, const double *b, double *out)
{
    const int nn[3] = {n[0], n[1], n[2]};
    const int cap = nn[0] + nn[1] + nn[2] + 8;
#pragma omp parallel
    {
        double *alpha = malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n_rays; ++r)
            out[r] = one_ray(vol, nn, h, o, a + 3 * r, b + 3 * r, alpha);
        free(alpha);
    }
    return 0;
}
