/*
 * oracle/edt_oracle.c -- CPU oracle for the truncated squared Euclidean
 * distance transform.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the benchmark's CPU-baseline leg call it; the product library never
 * links, loads or calls it, and it shares no code with the HIP path.
 *
 * What is computed (VDB-EDT paper, section III, Eq. 1 with the limited
 * transform of the same section): for every voxel x of an nx*ny*nz grid
 *
 *     s(x) = min( D, min over occupied y of |x - y|^2 ),   D = d_max^2,
 *
 * with |.|^2 the squared Euclidean distance in voxel units (the distance
 * measure the paper names first), min over an empty set = +infinity, and the
 * value D standing for every cell beyond the transform radius (the paper's
 * background value d_max of Initialize, read as a squared distance).
 * Occupied voxels get 0.  Only voxels inside the grid are obstacles.
 *
 * Layout: occ and out are x-fastest, index x + nx*(y + ny*z); occ nonzero =
 * occupied.  All arithmetic is exact int32.
 *
 * Three evaluations of the same definition:
 *   oracle_edt_bruteforce  scatters |x - y|^2 from every obstacle y over the
 *                          cube |x - y|_inf <= d_max (terms outside it are
 *                          > D and cannot change min(D, .)).
 *   oracle_edt_points      the definition at listed voxels only, scanning the
 *                          same cube around each listed voxel.
 *   oracle_edt_separable   |x - y|^2 = dx^2 + dy^2 + dz^2, so the minimum over
 *                          y can be taken one axis at a time (the separable
 *                          form of the global transform the paper cites in
 *                          section I); each axis pass is the plain windowed
 *                          minimum  g'(i) = min_{|j| <= d_max} g(i + j) + j^2.
 *                          Pinned against the brute force by the tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF (1 << 28)  /* "no obstacle"; INF + 3 * 255^2 fits in int32 */

static int check_args(int nx, int ny, int nz, int dmax) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return -1;
    if (dmax < 1 || dmax > 4095) return -1;
    return 0;
}

int oracle_edt_bruteforce(const uint8_t* occ, int nx, int ny, int nz, int dmax,
                          int32_t* out) {
    if (check_args(nx, ny, nz, dmax)) return -1;
    const int64_t n = (int64_t)nx * ny * nz;
    const int32_t D = dmax * dmax;
    for (int64_t i = 0; i < n; ++i) out[i] = D;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!occ[x + (int64_t)nx * (y + (int64_t)ny * z)]) continue;
                int z0 = z - dmax < 0 ? 0 : z - dmax, z1 = z + dmax >= nz ? nz - 1 : z + dmax;
                int y0 = y - dmax < 0 ? 0 : y - dmax, y1 = y + dmax >= ny ? ny - 1 : y + dmax;
                int x0 = x - dmax < 0 ? 0 : x - dmax, x1 = x + dmax >= nx ? nx - 1 : x + dmax;
                for (int zz = z0; zz <= z1; ++zz)
                    for (int yy = y0; yy <= y1; ++yy)
                        for (int xx = x0; xx <= x1; ++xx) {
                            int32_t d2 = (xx - x) * (xx - x) + (yy - y) * (yy - y) +
                                         (zz - z) * (zz - z);
                            int32_t* o = &out[xx + (int64_t)nx * (yy + (int64_t)ny * zz)];
                            if (d2 < *o) *o = d2;
                        }
            }
    return 0;
}

int oracle_edt_points(const uint8_t* occ, int nx, int ny, int nz, int dmax,
                      const int32_t* xyz, int64_t npts, int32_t* out) {
    if (check_args(nx, ny, nz, dmax)) return -1;
    const int32_t D = dmax * dmax;
    for (int64_t p = 0; p < npts; ++p) {
        int x = xyz[3 * p], y = xyz[3 * p + 1], z = xyz[3 * p + 2];
        int32_t best = D;
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) {
            out[p] = D;
            continue;
        }
        for (int zz = z - dmax; zz <= z + dmax; ++zz) {
            if (zz < 0 || zz >= nz) continue;
            for (int yy = y - dmax; yy <= y + dmax; ++yy) {
                if (yy < 0 || yy >= ny) continue;
                for (int xx = x - dmax; xx <= x + dmax; ++xx) {
                    if (xx < 0 || xx >= nx) continue;
                    if (!occ[xx + (int64_t)nx * (yy + (int64_t)ny * zz)]) continue;
                    int32_t d2 = (xx - x) * (xx - x) + (yy - y) * (yy - y) + (zz - z) * (zz - z);
                    if (d2 < best) best = d2;
                }
            }
        }
        out[p] = best;
    }
    return 0;
}

/* g1(x,y,z) = min over |i| <= dmax with occ(x+i,y,z) of i^2 (INF if none). */
static void pass_x(const uint8_t* occ, int nx, int ny, int nz, int dmax, int32_t* g1) {
    #pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < (int64_t)ny * nz; ++row) {
        const uint8_t* o = occ + row * nx;
        int32_t* g = g1 + row * nx;
        for (int x = 0; x < nx; ++x) {
            int32_t best = ORACLE_INF;
            for (int i = -dmax; i <= dmax; ++i) {
                int xx = x + i;
                if (xx < 0 || xx >= nx) continue;
                if (o[xx] && i * i < best) best = i * i;
            }
            g[x] = best;
        }
    }
}

/* g2(x,y,z) = min over |j| <= dmax of g1(x,y+j,z) + j^2. */
static void pass_y(const int32_t* g1, int nx, int ny, int nz, int dmax, int32_t* g2) {
    #pragma omp parallel for schedule(static)
    for (int64_t zy = 0; zy < (int64_t)ny * nz; ++zy) {
        int64_t z = zy / ny, y = zy % ny;
        int32_t* dst = g2 + (z * ny + y) * nx;
        for (int x = 0; x < nx; ++x) dst[x] = ORACLE_INF;
        for (int j = -dmax; j <= dmax; ++j) {
            int64_t yy = y + j;
            if (yy < 0 || yy >= ny) continue;
            const int32_t* src = g1 + (z * ny + yy) * nx;
            int32_t jj = j * j;
            for (int x = 0; x < nx; ++x) {
                int32_t v = src[x] + jj;
                if (v < dst[x]) dst[x] = v;
            }
        }
    }
}

/* s(x,y,z) = min(D, min over |k| <= dmax of g2(x,y,z+k) + k^2). */
static void pass_z(const int32_t* g2, int nx, int ny, int nz, int dmax, int32_t* s) {
    const int32_t D = dmax * dmax;
    #pragma omp parallel for schedule(static)
    for (int64_t zy = 0; zy < (int64_t)ny * nz; ++zy) {
        int64_t z = zy / ny, y = zy % ny;
        int32_t* dst = s + (z * ny + y) * nx;
        for (int x = 0; x < nx; ++x) dst[x] = D;
        for (int k = -dmax; k <= dmax; ++k) {
            int64_t zz = z + k;
            if (zz < 0 || zz >= nz) continue;
            const int32_t* src = g2 + (zz * ny + y) * nx;
            int32_t kk = k * k;
            for (int x = 0; x < nx; ++x) {
                int32_t v = src[x] + kk;
                if (v < dst[x]) dst[x] = v;
            }
        }
    }
}

int oracle_edt_separable(const uint8_t* occ, int nx, int ny, int nz, int dmax,
                         int32_t* out) {
    if (check_args(nx, ny, nz, dmax)) return -1;
    const int64_t n = (int64_t)nx * ny * nz;
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!tmp) return -2;
    pass_x(occ, nx, ny, nz, dmax, out);   /* out <- g1 */
    pass_y(out, nx, ny, nz, dmax, tmp);   /* tmp <- g2 */
    pass_z(tmp, nx, ny, nz, dmax, out);   /* out <- s  */
    free(tmp);
    return 0;
}

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the separable oracle uses (1 without OpenMP). */
int oracle_threads(int set) {
#ifdef _OPENMP
    if (set > 0) omp_set_num_threads(set);
    return omp_get_max_threads();
#else
    (void)set;
    return 1;
#endif
}
