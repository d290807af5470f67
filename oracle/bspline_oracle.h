/*
 * FP64 CPU oracle for periodic tricubic B-spline orbital evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may build, load or call this code.  It
 * shares no source, header, table or helper with the GPU library; the two
 * meet only through the seeded input generator.
 *
 * What it computes (paper: "QMC and B-spline-based SPOs", Eq. SplineFunc and
 * Eq. TricubicValue): for each position r and spline n,
 *
 *   phi_n(r) = sum_{a,b,c=0..3} Bx_a By_b Bz_c p[ix0-1+a][iy0-1+b][iz0-1+c][n]
 *
 * with i0 = floor(x/Delta) per dimension and B the centered uniform cubic
 * B-spline evaluated at t+1-m.  Gradient and Hessian are derivatives with
 * respect to the Cartesian position (section "Baseline and miniQMC", VGH
 * description), the Laplacian is the Hessian trace.
 *
 * Conventions shared with the library contract (restated here, not shared):
 *   coefficients  unpadded [nx][ny][nz][ncoef] (periodic), or, with
 *                 padded != 0, [nx+3][ny+3][nz+3][ncoef] read as-is;
 *   positions     [3][npos] FP64 (x row, y row, z row);
 *   outputs       FP64, v[p*ldo+n], g[(p*3+d)*ldo+n], l[p*ldo+n],
 *                 h[(p*6+k)*ldo+n] with k = xx,xy,xz,yy,yz,zz.
 *   A non-finite position yields NaN in every output of that position.
 */
#ifndef BSPLINE_ORACLE_H
#define BSPLINE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_V = 0, ORACLE_VGL = 1, ORACLE_VGH = 2 };
enum { ORACLE_COEF_F64 = 0, ORACLE_COEF_F32 = 1 };

/* Centered cubic B-spline and its first two derivatives at s. */
void oracle_basis(double s, double* b, double* db, double* d2b);

/* The four 1-D weights of a cell at fraction t in [0,1): w[m] = B(t+1-m),
 * dw[m] = B'(t+1-m)/delta, d2w[m] = B''(t+1-m)/delta^2.                   */
void oracle_weights(double t, double delta, double w[4], double dw[4], double d2w[4]);

/* Periodic cell location: returns 0 and sets *i0, *t for a finite x with
 * |x/delta| < 2^50; returns -1 otherwise.                                   */
int oracle_locate(double x, double box_len, int n, int* i0, double* t);

/* Evaluate.  kind is ORACLE_V/VGL/VGH; g and l/h may be NULL when the kind
 * does not produce them.  Returns 0, or -1 on bad arguments or a finite
 * position too far from the origin to keep any fraction bits.             */
int oracle_eval(int kind, int nx, int ny, int nz, int64_t ncoef,
                const void* coef, int coef_dtype, int padded,
                const double box[3], int64_t npos, const double* pos,
                double* v, double* g, double* l, double* h, int64_t ldo);

/* Brute force over every grid point and enough periodic images, with no
 * cell index and no wrap (tiny tables only).  Always produces V, G, L and H
 * (pass arrays for all).  Periodic unpadded f64 coefficients.              */
int oracle_eval_bruteforce(int nx, int ny, int nz, int64_t ncoef,
                           const double* coef, const double box[3],
                           int64_t npos, const double* pos,
                           double* v, double* g, double* l, double* h, int64_t ldo);

/* Determinant ratios (paper, "QMC and B-spline-based SPOs": the ratio of
 * determinants after a one-electron move and its gradient are sums over the
 * orbitals of phi_n(r_e), resp. grad phi_n(r_e), times the inverse-matrix
 * entry of (n, e)).  For each position p and output component c of `kind`
 * (same components and order as oracle_eval: V -> v; VGL -> v, gx, gy, gz,
 * l; VGH -> v, gx, gy, gz, hxx, hxy, hxz, hyy, hyz, hzz):
 *   out[p*ncomp + c] = sum_n X_{c,n}(r_p) * ainv[p*ld_ainv + n]
 * ainv is FP64 [npos][ld_ainv].  Returns 0, or -1 as oracle_eval.         */
int oracle_eval_ratio(int kind, int nx, int ny, int nz, int64_t ncoef,
                      const void* coef, int coef_dtype, const double box[3],
                      int64_t npos, const double* pos, const double* ainv,
                      int64_t ld_ainv, double* out);

/* General periodic cell with vectors a_i = lattice[3i..3i+2] (rows of A).
 * Grid coordinates u_d = n_d (r A^-1)_d; the spline is evaluated in grid
 * units and its derivatives carried to Cartesian ones by the chain rule
 * (M = du/dr: g_r = M^T g_u, H_r = M^T H_u M, L = trace H_r).  Arguments
 * and outputs as oracle_eval.  Returns -1 also for a singular lattice.    */
int oracle_eval_lattice(int kind, int nx, int ny, int nz, int64_t ncoef,
                        const void* coef, int coef_dtype, int padded,
                        const double lattice[9], int64_t npos, const double* pos,
                        double* v, double* g, double* l, double* h, int64_t ldo);

/* Interpolating coefficients: the unpadded periodic coefficients c
 * [nx][ny][nz][ncoef] whose spline takes the value values[i][j][k][n] at
 * grid point (i, j, k) (grid units; any cell).  Solves the circulant
 * tridiagonal system (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i] along each axis
 * with a dense inverse.  values and coefs may not overlap.  Returns 0, or
 * -1 on bad arguments.                                                     */
int oracle_fit_interpolating(int nx, int ny, int nz, int64_t ncoef, const double* values,
                             double* coefs);

/* Number of OpenMP threads an oracle_eval call uses. */
int oracle_num_threads(void);

/* Set that number (n > 0) for later calls on the calling thread. */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif

#endif
