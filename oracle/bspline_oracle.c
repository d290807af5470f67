/*
 * FP64 CPU oracle for periodic tricubic B-spline orbital evaluation.
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.
 *
 * Every function follows the paper's definition directly, in the paper's
 * order: locate the cell (Eq. SplineFunc: i = floor(x/Delta)), form the 1-D
 * weights, then sum the 4x4x4 tensor product (Eq. TricubicValue).  There is
 * no blocking or reordering beyond that definition.
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes):
 *  - basis (paper Fig. 2 is missing): the uniform cubic B-spline, written
 *    here as the centered function B(s) of de Boor's "Practical Guide to
 *    Splines", so the term for coefficient i0-1+m at fraction t is
 *    B(t+1-m);
 *  - index offset: the sum runs over i0-1 .. i0+2 (Eq. SplineFunc), and the
 *    unpadded table is periodic, so coefficient index (i0-1+m) mod n;
 *  - box: orthorhombic, Delta_d = L_d/n_d; positions wrap periodically;
 *  - derivatives are Cartesian (1/Delta, 1/Delta^2), Laplacian = trace H;
 *  - Hessian keeps the 6 upper-triangle components xx,xy,xz,yy,yz,zz;
 *  - outputs are overwritten, not accumulated into.
 */
#include "bspline_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void oracle_basis(double s, double* b, double* db, double* d2b)
{
    double a = fabs(s);
    double sg = (s < 0.0) ? -1.0 : 1.0;
    if (a < 1.0) {
        *b = 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        *db = sg * (-2.0 * a + 1.5 * a * a);
        *d2b = -2.0 + 3.0 * a;
    } else if (a < 2.0) {
        double r = 2.0 - a;
        *b = r * r * r / 6.0;
        *db = -sg * 0.5 * r * r;
        *d2b = r;
    } else {
        *b = 0.0;
        *db = 0.0;
        *d2b = 0.0;
    }
}

void oracle_weights(double t, double delta, double w[4], double dw[4], double d2w[4])
{
    for (int m = 0; m < 4; ++m) {
        double b, db, d2b;
        oracle_basis(t + 1.0 - m, &b, &db, &d2b);
        w[m] = b;
        dw[m] = db / delta;
        d2w[m] = d2b / (delta * delta);
    }
}

int oracle_locate(double x, double box_len, int n, int* i0, double* t)
{
    double delta = box_len / n;
    double u = x / delta;
    if (!isfinite(u) || fabs(u) >= 1125899906842624.0 /* 2^50 */)
        return -1;
    /* periodic wrap into [0, n) */
    u = u - n * floor(u / n);
    if (u < 0.0)
        u += n;
    int i = (int)floor(u);
    if (i >= n) { /* u rounded up to n: it is the image of 0 */
        i = 0;
        u = 0.0;
    }
    *i0 = i;
    *t = u - i;
    return 0;
}

static inline double coef_at(const void* coef, int dtype, int64_t idx)
{
    return dtype == ORACLE_COEF_F32 ? (double)((const float*)coef)[idx]
                                    : ((const double*)coef)[idx];
}

static inline int wrap_index(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static void fill_nan(int kind, int64_t p, int64_t ncoef, int64_t ldo,
                     double* v, double* g, double* l, double* h)
{
    double q = NAN;
    for (int64_t n = 0; n < ncoef; ++n) {
        v[p * ldo + n] = q;
        if (kind >= ORACLE_VGL)
            for (int d = 0; d < 3; ++d) g[(p * 3 + d) * ldo + n] = q;
        if (kind == ORACLE_VGL) l[p * ldo + n] = q;
        if (kind == ORACLE_VGH)
            for (int k = 0; k < 6; ++k) h[(p * 6 + k) * ldo + n] = q;
    }
}

int oracle_eval(int kind, int nx, int ny, int nz, int64_t ncoef,
                const void* coef, int coef_dtype, int padded,
                const double box[3], int64_t npos, const double* pos,
                double* v, double* g, double* l, double* h, int64_t ldo)
{
    if (kind < ORACLE_V || kind > ORACLE_VGH || nx <= 0 || ny <= 0 || nz <= 0 ||
        ncoef <= 0 || npos < 0 || ldo < ncoef || !coef || (npos > 0 && (!pos || !v)))
        return -1;
    if (kind >= ORACLE_VGL && npos > 0 && !g) return -1;
    if (kind == ORACLE_VGL && npos > 0 && !l) return -1;
    if (kind == ORACLE_VGH && npos > 0 && !h) return -1;
    const int dims[3] = {nx, ny, nz};
    const double L[3] = {box ? box[0] : 1.0, box ? box[1] : 1.0, box ? box[2] : 1.0};
    const int64_t sy = padded ? (int64_t)(nz + 3) : (int64_t)nz;
    const int64_t sx = padded ? (int64_t)(ny + 3) * sy : (int64_t)ny * sy;
    int status = 0;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npos; ++p) {
        int i0[3];
        double t[3], w[3][4], dw[3][4], d2w[3][4];
        int bad = 0;
        for (int d = 0; d < 3; ++d) {
            double x = pos[d * npos + p];
            if (!isfinite(x)) { bad = 1; break; }
            if (oracle_locate(x, L[d], dims[d], &i0[d], &t[d]) != 0) { bad = 2; break; }
            oracle_weights(t[d], L[d] / dims[d], w[d], dw[d], d2w[d]);
        }
        if (bad == 1) { fill_nan(kind, p, ncoef, ldo, v, g, l, h); continue; }
        if (bad == 2) {
#pragma omp atomic write
            status = -1;
            continue;
        }

        /* zero this position's outputs, then sum the 64 tensor-product terms */
        for (int64_t n = 0; n < ncoef; ++n) {
            v[p * ldo + n] = 0.0;
            if (kind >= ORACLE_VGL)
                for (int d = 0; d < 3; ++d) g[(p * 3 + d) * ldo + n] = 0.0;
            if (kind == ORACLE_VGL) l[p * ldo + n] = 0.0;
            if (kind == ORACLE_VGH)
                for (int k = 0; k < 6; ++k) h[(p * 6 + k) * ldo + n] = 0.0;
        }
        for (int a = 0; a < 4; ++a) {
            int ix = padded ? i0[0] + a : wrap_index(i0[0] - 1 + a, nx);
            for (int b = 0; b < 4; ++b) {
                int iy = padded ? i0[1] + b : wrap_index(i0[1] - 1 + b, ny);
                for (int c = 0; c < 4; ++c) {
                    int iz = padded ? i0[2] + c : wrap_index(i0[2] - 1 + c, nz);
                    const int64_t row = ((int64_t)ix * sx + (int64_t)iy * sy + iz) * ncoef;
                    /* weight of this term for each output component */
                    const double wv = w[0][a] * w[1][b] * w[2][c];
                    const double wgx = dw[0][a] * w[1][b] * w[2][c];
                    const double wgy = w[0][a] * dw[1][b] * w[2][c];
                    const double wgz = w[0][a] * w[1][b] * dw[2][c];
                    const double whxx = d2w[0][a] * w[1][b] * w[2][c];
                    const double whxy = dw[0][a] * dw[1][b] * w[2][c];
                    const double whxz = dw[0][a] * w[1][b] * dw[2][c];
                    const double whyy = w[0][a] * d2w[1][b] * w[2][c];
                    const double whyz = w[0][a] * dw[1][b] * dw[2][c];
                    const double whzz = w[0][a] * w[1][b] * d2w[2][c];
                    for (int64_t n = 0; n < ncoef; ++n) {
                        const double cf = coef_at(coef, coef_dtype, row + n);
                        v[p * ldo + n] += wv * cf;
                        if (kind >= ORACLE_VGL) {
                            g[(p * 3 + 0) * ldo + n] += wgx * cf;
                            g[(p * 3 + 1) * ldo + n] += wgy * cf;
                            g[(p * 3 + 2) * ldo + n] += wgz * cf;
                        }
                        if (kind == ORACLE_VGL)
                            l[p * ldo + n] += (whxx + whyy + whzz) * cf;
                        if (kind == ORACLE_VGH) {
                            h[(p * 6 + 0) * ldo + n] += whxx * cf;
                            h[(p * 6 + 1) * ldo + n] += whxy * cf;
                            h[(p * 6 + 2) * ldo + n] += whxz * cf;
                            h[(p * 6 + 3) * ldo + n] += whyy * cf;
                            h[(p * 6 + 4) * ldo + n] += whyz * cf;
                            h[(p * 6 + 5) * ldo + n] += whzz * cf;
                        }
                    }
                }
            }
        }
    }
    return status;
}

int oracle_eval_ratio(int kind, int nx, int ny, int nz, int64_t ncoef,
                      const void* coef, int coef_dtype, const double box[3],
                      int64_t npos, const double* pos, const double* ainv,
                      int64_t ld_ainv, double* out)
{
    if (kind < ORACLE_V || kind > ORACLE_VGH || npos < 0 || ncoef <= 0 || ld_ainv < ncoef ||
        (npos > 0 && (!pos || !ainv || !out)))
        return -1;
    const int ncomp = kind == ORACLE_V ? 1 : (kind == ORACLE_VGL ? 5 : 10);
    if (npos == 0) return 0;
    /* first the orbitals and their derivatives (Eq. TricubicValue) ... */
    double* v = (double*)malloc(sizeof(double) * (size_t)(npos * ncoef));
    double* g = kind >= ORACLE_VGL ? (double*)malloc(sizeof(double) * (size_t)(npos * 3 * ncoef)) : NULL;
    double* l = kind == ORACLE_VGL ? (double*)malloc(sizeof(double) * (size_t)(npos * ncoef)) : NULL;
    double* h = kind == ORACLE_VGH ? (double*)malloc(sizeof(double) * (size_t)(npos * 6 * ncoef)) : NULL;
    int rc = -1;
    if (v && (kind < ORACLE_VGL || g) && (kind != ORACLE_VGL || l) && (kind != ORACLE_VGH || h))
        rc = oracle_eval(kind, nx, ny, nz, ncoef, coef, coef_dtype, 0, box, npos, pos, v, g, l,
                         h, ncoef);
    /* ... then the ratio sums over the orbitals */
    if (rc == 0) {
        for (int64_t p = 0; p < npos; ++p) {
            const double* a = ainv + p * ld_ainv;
            for (int c = 0; c < ncomp; ++c) {
                const double* x;
                if (c == 0) x = v + p * ncoef;
                else if (c <= 3) x = g + (p * 3 + (c - 1)) * ncoef;
                else if (kind == ORACLE_VGL) x = l + p * ncoef;
                else x = h + (p * 6 + (c - 4)) * ncoef;
                double sum = 0.0;
                for (int64_t n = 0; n < ncoef; ++n) sum += x[n] * a[n];
                out[p * ncomp + c] = sum;
            }
        }
    }
    free(v);
    free(g);
    free(l);
    free(h);
    return rc;
}

/* Inverse of a 3x3 matrix by Gauss-Jordan elimination with partial
 * pivoting; returns -1 if it is singular. */
static int invert3(const double a_in[9], double inv[9])
{
    double a[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j)
            a[i][j] = j < 3 ? a_in[3 * i + j] : (j - 3 == i ? 1.0 : 0.0);
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (!(fabs(a[piv][c]) > 0.0)) return -1;
        for (int j = 0; j < 6; ++j) {
            double tmp = a[c][j];
            a[c][j] = a[piv][j];
            a[piv][j] = tmp;
        }
        double d = a[c][c];
        for (int j = 0; j < 6; ++j) a[c][j] /= d;
        for (int r = 0; r < 3; ++r) {
            if (r == c) continue;
            double f = a[r][c];
            for (int j = 0; j < 6; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) inv[3 * i + j] = a[i][j + 3];
    return 0;
}

int oracle_eval_lattice(int kind, int nx, int ny, int nz, int64_t ncoef,
                        const void* coef, int coef_dtype, int padded,
                        const double lattice[9], int64_t npos, const double* pos,
                        double* v, double* g, double* l, double* h, int64_t ldo)
{
    if (!lattice || kind < ORACLE_V || kind > ORACLE_VGH || npos < 0 || ncoef <= 0 ||
        ldo < ncoef || (npos > 0 && (!pos || !v)))
        return -1;
    if (kind >= ORACLE_VGL && npos > 0 && !g) return -1;
    if (kind == ORACLE_VGL && npos > 0 && !l) return -1;
    if (kind == ORACLE_VGH && npos > 0 && !h) return -1;
    double ainv[9];
    if (invert3(lattice, ainv) != 0) return -1;
    const int dims[3] = {nx, ny, nz};
    /* M[d][a] = du_d/dr_a = n_d (A^-1)[a][d] */
    double M[3][3];
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 3; ++a) M[d][a] = dims[d] * ainv[3 * a + d];
    if (npos == 0) return 0;
    /* 1. grid coordinates of every position */
    double* u = (double*)malloc(sizeof(double) * 3 * (size_t)npos);
    double* gu = (double*)malloc(sizeof(double) * 3 * (size_t)(npos * ncoef));
    double* hu = (double*)malloc(sizeof(double) * 6 * (size_t)(npos * ncoef));
    int rc = -1;
    if (u && gu && hu) {
        for (int64_t p = 0; p < npos; ++p)
            for (int d = 0; d < 3; ++d)
                u[d * npos + p] = M[d][0] * pos[p] + M[d][1] * pos[npos + p] +
                                  M[d][2] * pos[2 * npos + p];
        /* 2. the spline in grid units (a box of n_d cells of unit width) */
        const double unit_box[3] = {nx, ny, nz};
        rc = oracle_eval(kind == ORACLE_V ? ORACLE_V : ORACLE_VGH, nx, ny, nz, ncoef, coef,
                         coef_dtype, padded, unit_box, npos, u, v, gu, NULL, hu, ncoef);
    }
    /* 3. chain rule to Cartesian derivatives */
    if (rc == 0 && kind >= ORACLE_VGL) {
        static const int hrow[6] = {0, 0, 0, 1, 1, 2}, hcol[6] = {0, 1, 2, 1, 2, 2};
        for (int64_t p = 0; p < npos; ++p)
            for (int64_t n = 0; n < ncoef; ++n) {
                double G[3], H[3][3];
                for (int d = 0; d < 3; ++d) G[d] = gu[(p * 3 + d) * ncoef + n];
                for (int k = 0; k < 6; ++k) {
                    double x = hu[(p * 6 + k) * ncoef + n];
                    H[hrow[k]][hcol[k]] = x;
                    H[hcol[k]][hrow[k]] = x;
                }
                for (int a = 0; a < 3; ++a) {
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d) s += M[d][a] * G[d];
                    g[(p * 3 + a) * ldo + n] = s;
                }
                double Hr[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double s = 0.0;
                        for (int d = 0; d < 3; ++d)
                            for (int e = 0; e < 3; ++e) s += M[d][a] * M[e][b] * H[d][e];
                        Hr[a][b] = s;
                    }
                if (kind == ORACLE_VGL)
                    l[p * ldo + n] = Hr[0][0] + Hr[1][1] + Hr[2][2];
                else
                    for (int k = 0; k < 6; ++k) h[(p * 6 + k) * ldo + n] = Hr[hrow[k]][hcol[k]];
            }
    }
    /* copy V to the caller's stride */
    if (rc == 0 && ldo != ncoef)
        for (int64_t p = npos - 1; p >= 0; --p)
            for (int64_t n = ncoef - 1; n >= 0; --n) v[p * ldo + n] = v[p * ncoef + n];
    free(u);
    free(gu);
    free(hu);
    return rc;
}

/* Periodic sum of the basis over images: S(u, m) = sum_k B(u - m - k n). */
static void image_sum(double u, int m, int n, double delta, double* s, double* ds, double* d2s)
{
    *s = *ds = *d2s = 0.0;
    long kmin = (long)floor((u - m - 2.0) / n) - 1;
    long kmax = (long)ceil((u - m + 2.0) / n) + 1;
    for (long k = kmin; k <= kmax; ++k) {
        double b, db, d2b;
        oracle_basis(u - m - (double)k * n, &b, &db, &d2b);
        *s += b;
        *ds += db / delta;
        *d2s += d2b / (delta * delta);
    }
}

int oracle_eval_bruteforce(int nx, int ny, int nz, int64_t ncoef,
                           const double* coef, const double box[3],
                           int64_t npos, const double* pos,
                           double* v, double* g, double* l, double* h, int64_t ldo)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || ncoef <= 0 || npos < 0 || ldo < ncoef || !coef)
        return -1;
    if (npos > 0 && (!pos || !v || !g || !l || !h)) return -1;
    const int dims[3] = {nx, ny, nz};
    const double L[3] = {box ? box[0] : 1.0, box ? box[1] : 1.0, box ? box[2] : 1.0};
    int maxn = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npos; ++p) {
        double* S = (double*)malloc(sizeof(double) * 9 * (size_t)maxn);
        for (int d = 0; d < 3; ++d) {
            double delta = L[d] / dims[d];
            double u = pos[d * npos + p] / delta;
            for (int m = 0; m < dims[d]; ++m)
                image_sum(u, m, dims[d], delta, &S[(d * 3 + 0) * maxn + m],
                          &S[(d * 3 + 1) * maxn + m], &S[(d * 3 + 2) * maxn + m]);
        }
#define SV(d, m) S[((d) * 3 + 0) * maxn + (m)]
#define SD(d, m) S[((d) * 3 + 1) * maxn + (m)]
#define SD2(d, m) S[((d) * 3 + 2) * maxn + (m)]
        for (int64_t n = 0; n < ncoef; ++n) {
            double acc[10] = {0};
            for (int mx = 0; mx < nx; ++mx)
                for (int my = 0; my < ny; ++my)
                    for (int mz = 0; mz < nz; ++mz) {
                        double c = coef[(((int64_t)mx * ny + my) * nz + mz) * ncoef + n];
                        acc[0] += c * SV(0, mx) * SV(1, my) * SV(2, mz);
                        acc[1] += c * SD(0, mx) * SV(1, my) * SV(2, mz);
                        acc[2] += c * SV(0, mx) * SD(1, my) * SV(2, mz);
                        acc[3] += c * SV(0, mx) * SV(1, my) * SD(2, mz);
                        acc[4] += c * SD2(0, mx) * SV(1, my) * SV(2, mz);
                        acc[5] += c * SD(0, mx) * SD(1, my) * SV(2, mz);
                        acc[6] += c * SD(0, mx) * SV(1, my) * SD(2, mz);
                        acc[7] += c * SV(0, mx) * SD2(1, my) * SV(2, mz);
                        acc[8] += c * SV(0, mx) * SD(1, my) * SD(2, mz);
                        acc[9] += c * SV(0, mx) * SV(1, my) * SD2(2, mz);
                    }
            v[p * ldo + n] = acc[0];
            for (int d = 0; d < 3; ++d) g[(p * 3 + d) * ldo + n] = acc[1 + d];
            for (int k = 0; k < 6; ++k) h[(p * 6 + k) * ldo + n] = acc[4 + k];
            l[p * ldo + n] = acc[4] + acc[7] + acc[9];
        }
#undef SV
#undef SD
#undef SD2
        free(S);
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Interpolating coefficients (paper, "QMC and B-spline-based SPOs": the
 * coefficients are the orbitals' interpolation tables).  Reading: the
 * periodic spline must take the given value at every grid point.  At a grid
 * point the fraction is 0 and the weights are B(1), B(0), B(-1), B(-2) =
 * 1/6, 2/3, 1/6, 0, so along one axis of n points the condition is the
 * circulant system
 *   (1/6) c[(i-1) mod n] + (4/6) c[i] + (1/6) c[(i+1) mod n] = f[i],
 * and in 3-D the Kronecker product of the three axis systems.  It is solved
 * here one axis at a time with the explicit inverse of each axis matrix
 * (Gauss-Jordan with partial pivoting), applied to every line. */
static int invert_n(int n, const double* a_in, double* inv)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)n * 2 * n);
    if (!a) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            a[i * 2 * n + j] = j < n ? a_in[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + c]) > fabs(a[piv * 2 * n + c])) piv = r;
        if (a[piv * 2 * n + c] == 0.0) {
            free(a);
            return -1;
        }
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = a[c * 2 * n + j];
                a[c * 2 * n + j] = a[piv * 2 * n + j];
                a[piv * 2 * n + j] = t;
            }
        double p = a[c * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * 2 * n + c];
            for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= f * a[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) inv[i * n + j] = a[i * 2 * n + n + j];
    free(a);
    return 0;
}

int oracle_fit_interpolating(int nx, int ny, int nz, int64_t ncoef, const double* values,
                             double* coefs)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || ncoef <= 0 || !values || !coefs) return -1;
    const int dims[3] = {nx, ny, nz};
    const int64_t total = (int64_t)nx * ny * nz * ncoef;
    double* cur = (double*)malloc(sizeof(double) * (size_t)total);
    double* nxt = (double*)malloc(sizeof(double) * (size_t)total);
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return -1;
    }
    memcpy(cur, values, sizeof(double) * (size_t)total);
    int rc = 0;
    for (int d = 0; d < 3 && rc == 0; ++d) {
        const int n = dims[d];
        double* A = (double*)calloc((size_t)n * n, sizeof(double));
        double* Ainv = (double*)malloc(sizeof(double) * (size_t)n * n);
        if (!A || !Ainv) rc = -1;
        if (rc == 0) {
            /* the axis matrix: value at grid point i of the periodic spline */
            for (int i = 0; i < n; ++i) {
                A[i * n + (i - 1 + n) % n] += 1.0 / 6.0;
                A[i * n + i] += 4.0 / 6.0;
                A[i * n + (i + 1) % n] += 1.0 / 6.0;
            }
            rc = invert_n(n, A, Ainv);
        }
        if (rc == 0) {
            /* element (i along axis d, rest) sits at outer*n*inner + i*inner + r */
            int64_t inner = ncoef;
            for (int e = d + 1; e < 3; ++e) inner *= dims[e];
            const int64_t outer = total / (inner * n);
#pragma omp parallel for collapse(2) schedule(static)
            for (int64_t o = 0; o < outer; ++o)
                for (int64_t r = 0; r < inner; ++r) {
                    const int64_t base = o * n * inner + r;
                    for (int i = 0; i < n; ++i) {
                        double s = 0.0;
                        for (int j = 0; j < n; ++j) s += Ainv[i * n + j] * cur[base + j * inner];
                        nxt[base + i * inner] = s;
                    }
                }
            double* t = cur;
            cur = nxt;
            nxt = t;
        }
        free(A);
        free(Ainv);
    }
    if (rc == 0) memcpy(coefs, cur, sizeof(double) * (size_t)total);
    free(cur);
    free(nxt);
    return rc;
}
