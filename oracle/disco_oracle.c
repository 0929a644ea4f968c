/*
 * FP64 CPU oracle for the dense registration objective of Ruehaak et al.,
 * "Estimation of Large Motion in Lung CT by Integrating Regularized Keypoint
 * Correspondences into Dense Deformable Registration" (IEEE TMI 2017, arXiv 1807.00467).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is compared against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header or table with the GPU library and includes nothing from it.
 *
 * Every quantity is computed in double precision by direct loops over the
 * definitions.  Loops over independent voxels / cells / nodes may run in parallel
 * (OpenMP); every sum that accumulates into a shared result (objective values and
 * the transpose P^T onto the control-grid nodes) is done serially in a fixed order.
 *
 * Discretisation (the paper defers it to cited work; the readings are listed in the
 * design notes):
 *   - voxel (i,j,k) has centre ((i+1/2)h_x, (j+1/2)h_y, (k+1/2)h_z); arrays are
 *     [k][j][i]; integrals use the midpoint rule, int f dx ~ h_x h_y h_z sum_v f(x_v);
 *   - the transformation is y(x) = x + u(x) with u a first-order B-spline (trilinear)
 *     on a regular node grid with m_a voxels per cell and axis (Sec. II-D1, II-D3);
 *     node p sits at p*H_a with H_a = m_a h_a; node fields are [3][nz][ny][nx];
 *   - image gradients are central differences with replicated borders;
 *   - the moving-image gradient is sampled at the warped point by trilinear
 *     interpolation with zero padding (eq. 1 reads grad M evaluated at y(x)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX3(i, j, k, nx, ny) ((((int64_t)(k)) * (ny) + (j)) * (nx) + (i))

/* ------------------------------------------------------------------------------ */
/* Image gradients: (grad I)_a[i] = (I[i+e_a] - I[i-e_a]) / (2 h_a), indices clamped */
/* to the volume (replicate border).  Needed by eq. 1 for both images.               */
/* Output layout: [N][3] doubles.                                                     */
/* ------------------------------------------------------------------------------ */
void or_image_gradient(const int64_t *n, const double *h, const float *img, double *out)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t im = i > 0 ? i - 1 : 0, ip = i < nx - 1 ? i + 1 : nx - 1;
                int64_t jm = j > 0 ? j - 1 : 0, jp = j < ny - 1 ? j + 1 : ny - 1;
                int64_t km = k > 0 ? k - 1 : 0, kp = k < nz - 1 ? k + 1 : nz - 1;
                double *o = out + 3 * IDX3(i, j, k, nx, ny);
                o[0] = ((double)img[IDX3(ip, j, k, nx, ny)] - (double)img[IDX3(im, j, k, nx, ny)]) / (2.0 * h[0]);
                o[1] = ((double)img[IDX3(i, jp, k, nx, ny)] - (double)img[IDX3(i, jm, k, nx, ny)]) / (2.0 * h[1]);
                o[2] = ((double)img[IDX3(i, j, kp, nx, ny)] - (double)img[IDX3(i, j, km, nx, ny)]) / (2.0 * h[2]);
            }
}

/* ------------------------------------------------------------------------------ */
/* Trilinear sampling of a 3-vector field g ([N][3]) at continuous voxel index      */
/* q = i0 + t (i0 integer, t in [0,1]), zero outside the volume.  Returns the value  */
/* G and the Jacobian JG[c][a] = dG_c/dy_a = (1/h_a) dG_c/dq_a of the trilinear     */
/* interpolant inside the cell with lower corner i0.                                 */
/* ------------------------------------------------------------------------------ */
static void sample_vec_at(const int64_t *n, const double *h, const double *g, const int64_t i0[3],
                          const double t[3], double G[3], double JG[3][3])
{
    for (int c = 0; c < 3; ++c) {
        G[c] = 0.0;
        JG[c][0] = JG[c][1] = JG[c][2] = 0.0;
    }
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                int64_t ii = i0[0] + cx, jj = i0[1] + cy, kk = i0[2] + cz;
                if (ii < 0 || ii >= n[0] || jj < 0 || jj >= n[1] || kk < 0 || kk >= n[2]) continue;
                double wx = cx ? t[0] : 1.0 - t[0], dwx = cx ? 1.0 : -1.0;
                double wy = cy ? t[1] : 1.0 - t[1], dwy = cy ? 1.0 : -1.0;
                double wz = cz ? t[2] : 1.0 - t[2], dwz = cz ? 1.0 : -1.0;
                const double *gv = g + 3 * IDX3(ii, jj, kk, n[0], n[1]);
                for (int c = 0; c < 3; ++c) {
                    G[c] += wx * wy * wz * gv[c];
                    JG[c][0] += dwx * wy * wz * gv[c] / h[0];
                    JG[c][1] += wx * dwy * wz * gv[c] / h[1];
                    JG[c][2] += wx * wy * dwz * gv[c] / h[2];
                }
            }
}

/* The cell of a sample point along one axis.  The continuous index is q = idx + uh   */
/* (idx the voxel index, uh = u/h the displacement in voxels); since idx is an integer, */
/* floor(q) = idx + floor(uh) exactly, and t = uh - floor(uh).  Splitting this way     */
/* keeps the displacement's own precision where |uh| is far below idx (forming idx + uh */
/* first would round such displacements away).  At an integer q the floor puts the     */
/* point in the cell to its right.  Far outside [-2, n+1] every corner is outside the   */
/* volume and the sample is zero whatever the cell, so uh is clamped there.            */
static void split_axis(int64_t idx, double uh, int64_t n, int64_t *i0, double *t)
{
    const double lo = -2.0 - (double)idx, hi = (double)n + 1.0 - (double)idx;
    if (!(uh > lo)) uh = lo;
    if (!(uh < hi)) uh = hi;
    const double f = floor(uh);
    *i0 = idx + (int64_t)f;
    *t = uh - f;
}

/* sample at continuous index q (any real): the cell is floor(q) */
static void sample_vec(const int64_t *n, const double *h, const double *g, const double q[3],
                       double G[3], double JG[3][3])
{
    int64_t i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) split_axis(0, q[a], n[a], &i0[a], &t[a]);
    sample_vec_at(n, h, g, i0, t, G, JG);
}

void or_sample_points(const int64_t *n, const double *h, const double *g, int64_t npts,
                      const double *q, double *G, double *JG)
{
    for (int64_t p = 0; p < npts; ++p) {
        double J[3][3];
        sample_vec(n, h, g, q + 3 * p, G + 3 * p, J);
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) JG[9 * p + 3 * c + a] = J[c][a];
    }
}

/* ------------------------------------------------------------------------------ */
/* Control grid -> voxel: trilinear weights of voxel index i along one axis.        */
/* Voxel i lies in cell c = i / m at local coordinate xi = (i mod m + 1/2)/m; it     */
/* takes weight (1 - xi) from node c and xi from node c + 1 (Sec. II-D1/II-D3:       */
/* first-order B-splines, trilinear interpolation of the deformation).              */
/* ------------------------------------------------------------------------------ */
static void axis_weights(int64_t i, int64_t m, int64_t *c, double *xi)
{
    *c = i / m;
    *xi = ((double)(i % m) + 0.5) / (double)m;
}

/* value of a node field f ([3][nz][ny][nx]) at voxel (i,j,k) */
static void interp_voxel(const int64_t *nn, const int64_t *m, const double *f, int64_t i, int64_t j,
                         int64_t k, double out[3])
{
    int64_t c[3];
    double xi[3];
    axis_weights(i, m[0], &c[0], &xi[0]);
    axis_weights(j, m[1], &c[1], &xi[1]);
    axis_weights(k, m[2], &c[2], &xi[2]);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    out[0] = out[1] = out[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? xi[0] : 1.0 - xi[0]) * (dy ? xi[1] : 1.0 - xi[1]) * (dz ? xi[2] : 1.0 - xi[2]);
                int64_t node = IDX3(c[0] + dx, c[1] + dy, c[2] + dz, nn[0], nn[1]);
                for (int a = 0; a < 3; ++a) out[a] += w * f[a * nnodes + node];
            }
}

/* P^T: add val[3] * phi_{v,node} (or phi^2 when squared) onto the 8 nodes of voxel (i,j,k) */
static void scatter_voxel(const int64_t *nn, const int64_t *m, double *f, int64_t i, int64_t j, int64_t k,
                          const double val[3], int squared)
{
    int64_t c[3];
    double xi[3];
    axis_weights(i, m[0], &c[0], &xi[0]);
    axis_weights(j, m[1], &c[1], &xi[1]);
    axis_weights(k, m[2], &c[2], &xi[2]);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? xi[0] : 1.0 - xi[0]) * (dy ? xi[1] : 1.0 - xi[1]) * (dz ? xi[2] : 1.0 - xi[2]);
                if (squared) w = w * w;
                int64_t node = IDX3(c[0] + dx, c[1] + dy, c[2] + dz, nn[0], nn[1]);
                for (int a = 0; a < 3; ++a) f[a * nnodes + node] += w * val[a];
            }
}

static void node_counts(const int64_t *n, const int64_t *m, int64_t nn[3])
{
    for (int a = 0; a < 3; ++a) nn[a] = n[a] / m[a] + 1;
}

/* displacement of voxel (i,j,k) in voxels of the moving image along each axis:    */
/* uh_a = (Pu)_a(x_v) / h_a, so that the warped point has continuous index q = idx + uh */
static void voxel_uh(const int64_t *nn, const int64_t *m, const double *h, const double *u, int64_t i,
                     int64_t j, int64_t k, double uh[3])
{
    double uv[3];
    interp_voxel(nn, m, u, i, j, k, uv);
    for (int a = 0; a < 3; ++a) uh[a] = uv[a] / h[a];
}

/* NGF quantities of one voxel (eq. 1) with the sample of grad T taken in the cell with */
/* lower corner i0 at fractions t: r, c = 1 - r^2 and s = JG^T dr/da.  b = grad R[v].  */
static void ngf_voxel(const int64_t *n, const double *h, double e2, const double *gT, const double *b,
                      const int64_t i0[3], const double t[3], double *r, double *c, double s[3])
{
    double a[3], JG[3][3];
    sample_vec_at(n, h, gT, i0, t, a, JG);
    const double Da = e2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    const double Db = e2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double P = e2 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double sq = sqrt(Da * Db);
    *r = P / sq;
    /* 1 - r^2 written without cancellation (Lagrange's identity for the 4-vectors
       (eta, a) and (eta, b)) */
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    const double cx = a[1] * b[2] - a[2] * b[1];
    const double cy = a[2] * b[0] - a[0] * b[2];
    const double cz = a[0] * b[1] - a[1] * b[0];
    *c = (e2 * (dx * dx + dy * dy + dz * dz) + cx * cx + cy * cy + cz * cz) / (Da * Db);
    double dr[3];
    for (int q = 0; q < 3; ++q) dr[q] = (b[q] - (P / Da) * a[q]) / sq;
    for (int q = 0; q < 3; ++q) s[q] = JG[0][q] * dr[0] + JG[1][q] * dr[1] + JG[2][q] * dr[2];
}

/* ------------------------------------------------------------------------------ */
/* NGF distance, eq. 1, with <f,g>_eta = eta^2 + f.g:                               */
/*   a = grad T(y(x_v)), b = grad R(x_v),                                            */
/*   r_v = <a,b>_eta / sqrt(|a|_eta^2 |b|_eta^2),   c_v = 1 - r_v^2,                 */
/*   D = h_x h_y h_z sum_v c_v.                                                      */
/* Derivatives with respect to the node displacements u (discretize-optimize,       */
/* Sec. II-D3):                                                                      */
/*   s_v = JG(y_v)^T dr/da,  dr/da = (b - (P/Da) a)/sqrt(Da Db),                     */
/*   grad D = -2 h^3 sum_v phi_v r_v s_v,                                            */
/*   Gauss-Newton matrix H_D = 2 h^3 J^T J with J_v = phi_v s_v^T (rank one per      */
/*   voxel); its diagonal is 2 h^3 sum_v phi_v^2 s_v^2.                              */
/* gR, gT are [N][3] gradient images; u is a node field.  g, diag (node fields),    */
/* s ([N][3]), r ([N]) and c ([N]) are optional outputs (NULL to skip).              */
/* Returns D.                                                                        */
/* ------------------------------------------------------------------------------ */
double or_ngf(const int64_t *n, const double *h, const int64_t *m, double eta, const double *gR,
              const double *gT, const double *u, double *g, double *diag, double *s_out, double *r_out,
              double *c_out)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double h3 = h[0] * h[1] * h[2];
    const double e2 = eta * eta;
    double *r = (double *)malloc(sizeof(double) * nvox);
    double *c = (double *)malloc(sizeof(double) * nvox);
    double *s = (double *)malloc(sizeof(double) * 3 * nvox);

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t v = IDX3(i, j, k, nx, ny);
                const int64_t idx[3] = {i, j, k};
                double uh[3], t[3];
                int64_t i0[3];
                /* y = x + u; continuous index q = y/h - 1/2 = index + u/h */
                voxel_uh(nn, m, h, u, i, j, k, uh);
                for (int a = 0; a < 3; ++a) split_axis(idx[a], uh[a], n[a], &i0[a], &t[a]);
                ngf_voxel(n, h, e2, gT, gR + 3 * v, i0, t, &r[v], &c[v], s + 3 * v);
            }

    double D = 0.0;
    for (int64_t v = 0; v < nvox; ++v) D += c[v];
    D *= h3;

    if (g) memset(g, 0, sizeof(double) * 3 * nnodes);
    if (diag) memset(diag, 0, sizeof(double) * 3 * nnodes);
    if (g || diag) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t v = IDX3(i, j, k, nx, ny);
                    double val[3];
                    if (g) {
                        for (int t = 0; t < 3; ++t) val[t] = -2.0 * h3 * r[v] * s[3 * v + t];
                        scatter_voxel(nn, m, g, i, j, k, val, 0);
                    }
                    if (diag) {
                        for (int t = 0; t < 3; ++t) val[t] = 2.0 * h3 * s[3 * v + t] * s[3 * v + t];
                        scatter_voxel(nn, m, diag, i, j, k, val, 1);
                    }
                }
    }
    if (s_out) memcpy(s_out, s, sizeof(double) * 3 * nvox);
    if (r_out) memcpy(r_out, r, sizeof(double) * nvox);
    if (c_out) memcpy(c_out, c, sizeof(double) * nvox);
    free(r);
    free(c);
    free(s);
    return D;
}

/* ------------------------------------------------------------------------------ */
/* Gauss-Newton product of the NGF term: H_D v = 2 h^3 sum_v phi_v s_v (s_v . (Pv)(x_v)) */
/* s is [N][3] from or_ngf at the linearisation point.                               */
/* ------------------------------------------------------------------------------ */
void or_ngf_hv(const int64_t *n, const double *h, const int64_t *m, const double *s, const double *v,
               double *Hv)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double h3 = h[0] * h[1] * h[2];
    double *w = (double *)malloc(sizeof(double) * nvox);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t vx = IDX3(i, j, k, nx, ny);
                double pv[3];
                interp_voxel(nn, m, v, i, j, k, pv);
                w[vx] = s[3 * vx] * pv[0] + s[3 * vx + 1] * pv[1] + s[3 * vx + 2] * pv[2];
            }
    memset(Hv, 0, sizeof(double) * 3 * nnodes);
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t vx = IDX3(i, j, k, nx, ny);
                double val[3];
                for (int t = 0; t < 3; ++t) val[t] = 2.0 * h3 * s[3 * vx + t] * w[vx];
                scatter_voxel(nn, m, Hv, i, j, k, val, 0);
            }
    free(w);
}

/* ------------------------------------------------------------------------------ */
/* Sample-cell ties.  Which cell of the moving-image grid holds a warped point is an  */
/* integer decision (the floor of q = idx + uh).  The trilinear interpolant is        */
/* continuous across cell faces, so the sampled value (and with it r, c and D) does   */
/* not depend on that decision, but its derivative JG jumps across a face: s, and     */
/* through s the gradient, GN diagonal and GN product, are one-sided there.  Where uh  */
/* lies within rounding of an integer, a single-precision evaluation of uh may land   */
/* on either side of the face, and both one-sided results are correct.                */
/*                                                                                    */
/* Bound.  uh_a is the trilinear interpolant of the 8 node values u_a of the voxel's   */
/* cell divided by h_a.  Evaluated in IEEE single precision by nested linear            */
/* interpolation (at most three levels of one subtraction and one multiply-add, then   */
/* one multiplication by a rounded 1/h_a), each rounding contributes at most           */
/* 2^-24 of a quantity bounded by 2 M_a (M_a = max over the 8 nodes of |u_a| / h_a),    */
/* so |uh_single - uh| < 12 * 2^-24 * M_a.  Axis a of a voxel is a tie when            */
/* dist(uh_a, nearest integer) < TIE_REL * M_a with TIE_REL = 2^-19 (32 * 2^-24, a     */
/* margin of more than two on the bound).  uh = 0 exactly from all-zero nodes          */
/* (M_a = 0) is never a tie.                                                          */
/*                                                                                    */
/* For every voxel with at least one tie axis the routine evaluates every other choice */
/* of cell on its tie axes (2^k - 1 alternatives for k tie axes; the other side of the */
/* face is taken at t = 1 on the left cell or t = 0 on the right cell) and returns,    */
/* per node, the sum over those voxels of the largest difference to the reference      */
/* (floor) choice, weighted like the quantity itself:                                 */
/*   ag   = sum_v phi_v   max |2h^3 (r' s'_c - r s_c)|            (gradient)          */
/*   adg  = sum_v phi_v^2 max |2h^3 (s'_c^2 - s_c^2)|             (GN diagonal)       */
/*   ahv  = sum_v phi_v   max |2h^3 (s'_c (s'.w) - s_c (s.w))|, w = (Pv)(x_v)  (GN v) */
/* and per voxel sdev = max |s'_c - s_c| (for the s vectors themselves).  Any of the   */
/* outputs may be NULL (v may be NULL when ahv is).  Returns the number of voxels with */
/* a tie.                                                                             */
/* ------------------------------------------------------------------------------ */
#define TIE_REL 1.9073486328125e-06 /* 2^-19 */

/* tie axes of voxel (i,j,k): bit a set when axis a is a tie; alt_i0/alt_t give the   */
/* other side of the face on those axes                                               */
static int tie_axes(const int64_t *nn, const int64_t *m, const int64_t *n, const double *h, const double *u,
                    int64_t i, int64_t j, int64_t k, const double uh[3], int64_t alt_i0[3], double alt_t[3])
{
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const int64_t idx[3] = {i, j, k};
    const int64_t c0 = i / m[0], c1 = j / m[1], c2 = k / m[2];
    int mask = 0;
    for (int a = 0; a < 3; ++a) {
        double M = 0.0;
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const double x = fabs(u[a * nnodes + IDX3(c0 + dx, c1 + dy, c2 + dz, nn[0], nn[1])]);
                    if (x > M) M = x;
                }
        M /= h[a];
        const double kint = nearbyint(uh[a]);
        if (!(fabs(uh[a] - kint) < TIE_REL * M)) continue;
        /* far outside the volume every corner is outside on both sides */
        if (idx[a] + kint < -2.0 || idx[a] + kint > (double)n[a] + 1.0) continue;
        mask |= 1 << a;
        if (uh[a] >= kint) { /* reference cell starts at the integer: other side is the left cell */
            alt_i0[a] = idx[a] + (int64_t)kint - 1;
            alt_t[a] = 1.0;
        } else { /* reference cell ends at the integer: other side is the right cell */
            alt_i0[a] = idx[a] + (int64_t)kint;
            alt_t[a] = 0.0;
        }
    }
    return mask;
}

int64_t or_ngf_ties(const int64_t *n, const double *h, const int64_t *m, double eta, const double *gR,
                    const double *gT, const double *u, const double *v, double *ag, double *adg, double *ahv,
                    double *sdev)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double h3 = h[0] * h[1] * h[2];
    const double e2 = eta * eta;
    uint8_t *flag = (uint8_t *)malloc((size_t)nvox);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double uh[3], at[3];
                int64_t ai[3];
                voxel_uh(nn, m, h, u, i, j, k, uh);
                flag[IDX3(i, j, k, nx, ny)] = (uint8_t)tie_axes(nn, m, n, h, u, i, j, k, uh, ai, at);
            }
    int64_t nt = 0;
    for (int64_t q = 0; q < nvox; ++q) nt += flag[q] != 0;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    nt = 0;
    for (int64_t q = 0; q < nvox; ++q)
        if (flag[q]) list[nt++] = q;
    double *dv = (double *)calloc((size_t)(12 * (nt > 0 ? nt : 1)), sizeof(double)); /* dg, dd, dh, ds */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < nt; ++e) {
        const int64_t vox = list[e];
        const int64_t i = vox % nx, j = (vox / nx) % ny, k = vox / (nx * ny);
        const int64_t idx[3] = {i, j, k};
        double uh[3], t0[3], at[3], w[3] = {0.0, 0.0, 0.0};
        int64_t i00[3], ai[3];
        voxel_uh(nn, m, h, u, i, j, k, uh);
        const int mask = tie_axes(nn, m, n, h, u, i, j, k, uh, ai, at);
        for (int a = 0; a < 3; ++a) split_axis(idx[a], uh[a], n[a], &i00[a], &t0[a]);
        if (v) interp_voxel(nn, m, v, i, j, k, w);
        double r0, c0, s0[3];
        ngf_voxel(n, h, e2, gT, gR + 3 * vox, i00, t0, &r0, &c0, s0);
        const double sw0 = s0[0] * w[0] + s0[1] * w[1] + s0[2] * w[2];
        double *o = dv + 12 * e;
        for (int combo = 1; combo < 8; ++combo) {
            if (combo & ~mask) continue;
            int64_t i1[3];
            double t1[3], r1, c1, s1[3];
            for (int a = 0; a < 3; ++a) {
                i1[a] = (combo >> a & 1) ? ai[a] : i00[a];
                t1[a] = (combo >> a & 1) ? at[a] : t0[a];
            }
            ngf_voxel(n, h, e2, gT, gR + 3 * vox, i1, t1, &r1, &c1, s1);
            const double sw1 = s1[0] * w[0] + s1[1] * w[1] + s1[2] * w[2];
            for (int q = 0; q < 3; ++q) {
                const double dg = fabs(2.0 * h3 * (r1 * s1[q] - r0 * s0[q]));
                const double dd = fabs(2.0 * h3 * (s1[q] * s1[q] - s0[q] * s0[q]));
                const double dh = fabs(2.0 * h3 * (s1[q] * sw1 - s0[q] * sw0));
                const double ds = fabs(s1[q] - s0[q]);
                if (dg > o[q]) o[q] = dg;
                if (dd > o[3 + q]) o[3 + q] = dd;
                if (dh > o[6 + q]) o[6 + q] = dh;
                if (ds > o[9 + q]) o[9 + q] = ds;
            }
        }
    }
    if (ag) memset(ag, 0, sizeof(double) * 3 * nnodes);
    if (adg) memset(adg, 0, sizeof(double) * 3 * nnodes);
    if (ahv) memset(ahv, 0, sizeof(double) * 3 * nnodes);
    if (sdev) memset(sdev, 0, sizeof(double) * 3 * nvox);
    for (int64_t e = 0; e < nt; ++e) {
        const int64_t vox = list[e];
        const int64_t i = vox % nx, j = (vox / nx) % ny, k = vox / (nx * ny);
        const double *o = dv + 12 * e;
        if (ag) scatter_voxel(nn, m, ag, i, j, k, o, 0);
        if (adg) scatter_voxel(nn, m, adg, i, j, k, o + 3, 1);
        if (ahv) scatter_voxel(nn, m, ahv, i, j, k, o + 6, 0);
        if (sdev)
            for (int q = 0; q < 3; ++q) sdev[3 * vox + q] = o[9 + q];
    }
    free(dv);
    free(list);
    free(flag);
    return nt;
}

/* ------------------------------------------------------------------------------ */
/* Curvature regulariser, eq. 5: S = 1/2 int sum_j |Lap(y_j - yhat_j)|^2 dx, with   */
/* Lap discretised on the node grid:                                                 */
/*   (L f)(p) = sum_a chi_a(p) (f(p-e_a) - 2 f(p) + f(p+e_a)) / H_a^2,               */
/*   chi_a(p) = 1 iff 1 <= p_a <= n_a - 2 (second differences vanish at the border), */
/* and the node-grid quadrature weight C_H = H_x H_y H_z:                            */
/*   S = 1/2 C_H sum_p sum_j ((L w_j)(p))^2,   w = u - uhat  (y - yhat = u - uhat).  */
/* Outputs: S, out = C_H L^T L w (the gradient, also the exact Hessian times w),     */
/* diag = C_H diag(L^T L) (same for each component; written for all 3).              */
/* Any output pointer may be NULL.  Returns S.                                       */
/* ------------------------------------------------------------------------------ */
static int chi(int64_t p, int64_t n) { return p >= 1 && p <= n - 2; }

double or_curvature(const int64_t *nn, const double *H, const double *w, double *out, double *diag)
{
    const int64_t nx = nn[0], ny = nn[1], nz = nn[2];
    const int64_t nnodes = nx * ny * nz;
    const double CH = H[0] * H[1] * H[2];
    const double ih2[3] = {1.0 / (H[0] * H[0]), 1.0 / (H[1] * H[1]), 1.0 / (H[2] * H[2])};
    double *Lw = (double *)malloc(sizeof(double) * 3 * nnodes);
    for (int j = 0; j < 3; ++j) {
        const double *f = w + j * nnodes;
        for (int64_t pz = 0; pz < nz; ++pz)
            for (int64_t py = 0; py < ny; ++py)
                for (int64_t px = 0; px < nx; ++px) {
                    double acc = 0.0;
                    int64_t p = IDX3(px, py, pz, nx, ny);
                    if (chi(px, nx)) acc += (f[p - 1] - 2.0 * f[p] + f[p + 1]) * ih2[0];
                    if (chi(py, ny)) acc += (f[p - nx] - 2.0 * f[p] + f[p + nx]) * ih2[1];
                    if (chi(pz, nz)) acc += (f[p - nx * ny] - 2.0 * f[p] + f[p + nx * ny]) * ih2[2];
                    Lw[j * nnodes + p] = acc;
                }
    }
    double S = 0.0;
    for (int64_t t = 0; t < 3 * nnodes; ++t) S += Lw[t] * Lw[t];
    S *= 0.5 * CH;

    if (out) {
        /* L^T applied row by row: row p of L has coefficient -2/H_a^2 at p and 1/H_a^2 at
           p -+ e_a for every axis a with chi_a(p) = 1 */
        memset(out, 0, sizeof(double) * 3 * nnodes);
        for (int j = 0; j < 3; ++j) {
            double *o = out + j * nnodes;
            const double *l = Lw + j * nnodes;
            for (int64_t pz = 0; pz < nz; ++pz)
                for (int64_t py = 0; py < ny; ++py)
                    for (int64_t px = 0; px < nx; ++px) {
                        int64_t p = IDX3(px, py, pz, nx, ny);
                        double val = l[p];
                        const int64_t stride[3] = {1, nx, nx * ny};
                        const int on[3] = {chi(px, nx), chi(py, ny), chi(pz, nz)};
                        for (int a = 0; a < 3; ++a) {
                            if (!on[a]) continue;
                            o[p - stride[a]] += CH * val * ih2[a];
                            o[p] += -2.0 * CH * val * ih2[a];
                            o[p + stride[a]] += CH * val * ih2[a];
                        }
                    }
        }
    }
    if (diag) {
        memset(diag, 0, sizeof(double) * nnodes);
        for (int64_t pz = 0; pz < nz; ++pz)
            for (int64_t py = 0; py < ny; ++py)
                for (int64_t px = 0; px < nx; ++px) {
                    int64_t p = IDX3(px, py, pz, nx, ny);
                    const int64_t stride[3] = {1, nx, nx * ny};
                    const int on[3] = {chi(px, nx), chi(py, ny), chi(pz, nz)};
                    double centre = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        if (!on[a]) continue;
                        centre += -2.0 * ih2[a];
                        diag[p - stride[a]] += ih2[a] * ih2[a];
                        diag[p + stride[a]] += ih2[a] * ih2[a];
                    }
                    diag[p] += centre * centre;
                }
        for (int64_t p = 0; p < nnodes; ++p) diag[p] *= CH;
        memcpy(diag + nnodes, diag, sizeof(double) * nnodes);
        memcpy(diag + 2 * nnodes, diag, sizeof(double) * nnodes);
    }
    free(Lw);
    return S;
}

/* ------------------------------------------------------------------------------ */
/* Volume change control, eq. 7-9.                                                   */
/* psi(t) = (t-1)^2/t for t > 0, +inf otherwise.                                     */
/* On a cell with corners y_ijk (i,j,k in {0,1}), the trilinear map has             */
/*   dy/dxi_1 = sum_{jk} w_j w_k e1_jk,  e1_jk = y_1jk - y_0jk  (same for xi_2, xi_3), */
/* so by multilinearity of the determinant                                           */
/*   det grad y = sum_{a,b,c} alpha_abc(xi) d_abc,  d_abc = det[e1_a, e2_b, e3_c] / C, */
/* with C = H_x H_y H_z the cell volume and alpha_abc >= 0 summing to one: the 64    */
/* terms of eq. 8.  Eq. 9: Vhat = C sum_cells sum_abc psi(d_abc).                    */
/* Index conventions: a = (j,k) -> j + 2k for e1 = y_1jk - y_0jk,                    */
/*                    b = (i,k) -> i + 2k for e2 = y_i1k - y_i0k,                    */
/*                    c = (i,j) -> i + 2j for e3 = y_ij1 - y_ij0.                    */
/* Derivatives: dd_abc/dy_node = sum over the three edges of the term that contain  */
/* the node of (+-1) x (cross product of the other two edges) / C.                   */
/* Gauss-Newton matrix: C sum psi''(d) grad d grad d^T (psi'' = 2/t^3 > 0).          */
/* Outputs (any may be NULL): g = grad Vhat, diag = diagonal of the GN matrix,      */
/* Hv = GN matrix times v.  nfold counts terms with d <= 0; then Vhat = +inf and    */
/* the derivative outputs are left as computed from the terms with d > 0.            */
/* dminmax receives (min d, max d).  Returns Vhat.                                   */
/* ------------------------------------------------------------------------------ */
static double psi(double t) { return t > 0.0 ? (t - 1.0) * (t - 1.0) / t : INFINITY; }
static double dpsi(double t) { return 1.0 - 1.0 / (t * t); }
static double d2psi(double t) { return 2.0 / (t * t * t); }

static void cross3(const double *x, const double *y, double *o)
{
    o[0] = x[1] * y[2] - x[2] * y[1];
    o[1] = x[2] * y[0] - x[0] * y[2];
    o[2] = x[0] * y[1] - x[1] * y[0];
}
static double dot3(const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; }

/* corner (i,j,k) of cell (cx,cy,cz): position X + u */
static void cell_corners(const int64_t *nn, const double *H, const double *u, int64_t cx, int64_t cy,
                         int64_t cz, double y[8][3], int64_t node[8])
{
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) {
                int corner = i + 2 * j + 4 * k;
                int64_t p = IDX3(cx + i, cy + j, cz + k, nn[0], nn[1]);
                node[corner] = p;
                y[corner][0] = (double)(cx + i) * H[0] + (u ? u[p] : 0.0);
                y[corner][1] = (double)(cy + j) * H[1] + (u ? u[nnodes + p] : 0.0);
                y[corner][2] = (double)(cz + k) * H[2] + (u ? u[2 * nnodes + p] : 0.0);
            }
}

/* The 64 coefficients d_abc of one cell and their derivatives dd[abc][corner][comp] */
static void cell_terms(const double y[8][3], double C, double d[64], double dd[64][8][3])
{
    double e1[4][3], e2[4][3], e3[4][3];
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int t = 0; t < 3; ++t) e1[j + 2 * k][t] = y[1 + 2 * j + 4 * k][t] - y[0 + 2 * j + 4 * k][t];
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 2; ++i)
            for (int t = 0; t < 3; ++t) e2[i + 2 * k][t] = y[i + 2 + 4 * k][t] - y[i + 0 + 4 * k][t];
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i)
            for (int t = 0; t < 3; ++t) e3[i + 2 * j][t] = y[i + 2 * j + 4][t] - y[i + 2 * j][t];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                int l = a + 4 * b + 16 * c;
                double x23[3], x31[3], x12[3];
                cross3(e2[b], e3[c], x23);
                cross3(e3[c], e1[a], x31);
                cross3(e1[a], e2[b], x12);
                d[l] = dot3(e1[a], x23) / C;
                memset(dd[l], 0, sizeof(double) * 24);
                /* e1_a = y_{1,ja,ka} - y_{0,ja,ka} */
                int ja = a & 1, ka = a >> 1;
                int ib = b & 1, kb = b >> 1;
                int ic = c & 1, jc = c >> 1;
                for (int t = 0; t < 3; ++t) {
                    dd[l][1 + 2 * ja + 4 * ka][t] += x23[t] / C;
                    dd[l][0 + 2 * ja + 4 * ka][t] -= x23[t] / C;
                    dd[l][ib + 2 + 4 * kb][t] += x31[t] / C;
                    dd[l][ib + 0 + 4 * kb][t] -= x31[t] / C;
                    dd[l][ic + 2 * jc + 4][t] += x12[t] / C;
                    dd[l][ic + 2 * jc + 0][t] -= x12[t] / C;
                }
            }
}

double or_vcc(const int64_t *nn, const double *H, const double *u, const double *v, double *g, double *diag,
              double *Hv, int64_t *nfold, double *dminmax)
{
    const int64_t ncx = nn[0] - 1, ncy = nn[1] - 1, ncz = nn[2] - 1;
    const int64_t ncell = ncx * ncy * ncz;
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double C = H[0] * H[1] * H[2];
    /* per-cell results, combined serially afterwards */
    double *cV = (double *)malloc(sizeof(double) * ncell);
    int64_t *cF = (int64_t *)malloc(sizeof(int64_t) * ncell);
    double *cMin = (double *)malloc(sizeof(double) * ncell);
    double *cMax = (double *)malloc(sizeof(double) * ncell);
    double *cG = g ? (double *)malloc(sizeof(double) * ncell * 24) : NULL;
    double *cD = diag ? (double *)malloc(sizeof(double) * ncell * 24) : NULL;
    double *cH = Hv ? (double *)malloc(sizeof(double) * ncell * 24) : NULL;

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t cell = 0; cell < ncell; ++cell) {
        int64_t cx = cell % ncx, cy = (cell / ncx) % ncy, cz = cell / (ncx * ncy);
        double y[8][3];
        int64_t node[8];
        double d[64];
        double(*dd)[8][3] = malloc(sizeof(double) * 64 * 24);
        cell_corners(nn, H, u, cx, cy, cz, y, node);
        cell_terms(y, C, d, dd);
        double vv[8][3];
        if (cH)
            for (int q = 0; q < 8; ++q)
                for (int t = 0; t < 3; ++t) vv[q][t] = v[t * nnodes + node[q]];
        double V = 0.0, mn = INFINITY, mx = -INFINITY;
        int64_t folds = 0;
        double G[8][3] = {{0}}, Dg[8][3] = {{0}}, Hc[8][3] = {{0}};
        for (int l = 0; l < 64; ++l) {
            if (d[l] < mn) mn = d[l];
            if (d[l] > mx) mx = d[l];
            if (!(d[l] > 0.0)) {
                ++folds;
                continue;
            }
            V += C * psi(d[l]);
            double p1 = dpsi(d[l]), p2 = d2psi(d[l]);
            double jv = 0.0;
            if (cH)
                for (int q = 0; q < 8; ++q) jv += dot3(dd[l][q], vv[q]);
            for (int q = 0; q < 8; ++q)
                for (int t = 0; t < 3; ++t) {
                    G[q][t] += C * p1 * dd[l][q][t];
                    Dg[q][t] += C * p2 * dd[l][q][t] * dd[l][q][t];
                    Hc[q][t] += C * p2 * jv * dd[l][q][t];
                }
        }
        cV[cell] = folds ? INFINITY : V;
        cF[cell] = folds;
        cMin[cell] = mn;
        cMax[cell] = mx;
        if (cG) memcpy(cG + 24 * cell, G, sizeof(G));
        if (cD) memcpy(cD + 24 * cell, Dg, sizeof(Dg));
        if (cH) memcpy(cH + 24 * cell, Hc, sizeof(Hc));
        free(dd);
    }

    double V = 0.0, mn = INFINITY, mx = -INFINITY;
    int64_t folds = 0;
    if (g) memset(g, 0, sizeof(double) * 3 * nnodes);
    if (diag) memset(diag, 0, sizeof(double) * 3 * nnodes);
    if (Hv) memset(Hv, 0, sizeof(double) * 3 * nnodes);
    for (int64_t cell = 0; cell < ncell; ++cell) {
        V += cV[cell];
        folds += cF[cell];
        if (cMin[cell] < mn) mn = cMin[cell];
        if (cMax[cell] > mx) mx = cMax[cell];
        int64_t cx = cell % ncx, cy = (cell / ncx) % ncy, cz = cell / (ncx * ncy);
        for (int q = 0; q < 8; ++q) {
            int64_t p = IDX3(cx + (q & 1), cy + ((q >> 1) & 1), cz + (q >> 2), nn[0], nn[1]);
            for (int t = 0; t < 3; ++t) {
                if (g) g[t * nnodes + p] += cG[24 * cell + 3 * q + t];
                if (diag) diag[t * nnodes + p] += cD[24 * cell + 3 * q + t];
                if (Hv) Hv[t * nnodes + p] += cH[24 * cell + 3 * q + t];
            }
        }
    }
    if (nfold) *nfold = folds;
    if (dminmax) {
        dminmax[0] = mn;
        dminmax[1] = mx;
    }
    free(cV);
    free(cF);
    free(cMin);
    free(cMax);
    free(cG);
    free(cD);
    free(cH);
    return folds ? INFINITY : V;
}

/* 64 coefficients alpha_abc(xi) and d_abc of one cell, and the exact determinant of
   grad y at local coordinate xi (for the eq. 8 identity and the bound of eq. 9). */
void or_vcc_cell_expansion(const int64_t *nn, const double *H, const double *u, const int64_t *cell,
                           const double *xi, double *alpha, double *d, double *det_exact)
{
    double y[8][3];
    int64_t node[8];
    double(*dd)[8][3] = malloc(sizeof(double) * 64 * 24);
    const double C = H[0] * H[1] * H[2];
    cell_corners(nn, H, u, cell[0], cell[1], cell[2], y, node);
    cell_terms(y, C, d, dd);
    free(dd);
    double w1[2] = {1.0 - xi[0], xi[0]}, w2[2] = {1.0 - xi[1], xi[1]}, w3[2] = {1.0 - xi[2], xi[2]};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                /* beta_a(xi2, xi3) for e1_(j,k); beta'_b(xi1, xi3) for e2_(i,k); beta''_c(xi1, xi2) */
                double ba = w2[a & 1] * w3[a >> 1];
                double bb = w1[b & 1] * w3[b >> 1];
                double bc = w1[c & 1] * w2[c >> 1];
                alpha[a + 4 * b + 16 * c] = ba * bb * bc;
            }
    /* exact Jacobian of the trilinear map: columns dy/dxi_a / H_a */
    double Jm[3][3] = {{0}};
    for (int corner = 0; corner < 8; ++corner) {
        int i = corner & 1, j = (corner >> 1) & 1, k = corner >> 2;
        double d1 = (i ? 1.0 : -1.0) * w2[j] * w3[k];
        double d2 = w1[i] * (j ? 1.0 : -1.0) * w3[k];
        double d3 = w1[i] * w2[j] * (k ? 1.0 : -1.0);
        for (int t = 0; t < 3; ++t) {
            Jm[t][0] += d1 * y[corner][t] / H[0];
            Jm[t][1] += d2 * y[corner][t] / H[1];
            Jm[t][2] += d3 * y[corner][t] / H[2];
        }
    }
    *det_exact = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                 Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                 Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
}

/* ------------------------------------------------------------------------------ */
/* Keypoint penalty, eq. 10: K = sum_i |y(x_i) - y_KP(x_i)|^2,                     */
/* y(x_i) = x_i + (P u)(x_i), trilinear on the node grid: xi_a = x_a / H_a,          */
/* cell p_a = min(floor(xi_a), n_a - 2), t = xi_a - p_a.                             */
/* grad K = 2 P^T res;  Hessian 2 P^T P (exact);  diag = 2 sum_i phi_i(node)^2.      */
/* Keypoints must lie in the closed box [0, N_a h_a]; returns NAN otherwise.        */
/* ------------------------------------------------------------------------------ */
static int kp_weights(const int64_t *nn, const double *H, const double *x, int64_t node[8], double w[8])
{
    int64_t p[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double xi = x[a] / H[a];
        if (!(xi >= 0.0 && xi <= (double)(nn[a] - 1))) return 0;
        double f = floor(xi);
        if (f > (double)(nn[a] - 2)) f = (double)(nn[a] - 2);
        p[a] = (int64_t)f;
        t[a] = xi - f;
    }
    for (int q = 0; q < 8; ++q) {
        int i = q & 1, j = (q >> 1) & 1, k = q >> 2;
        node[q] = IDX3(p[0] + i, p[1] + j, p[2] + k, nn[0], nn[1]);
        w[q] = (i ? t[0] : 1.0 - t[0]) * (j ? t[1] : 1.0 - t[1]) * (k ? t[2] : 1.0 - t[2]);
    }
    return 1;
}

double or_keypoints(const int64_t *nn, const double *H, int64_t npts, const double *x, const double *tgt,
                    const double *u, const double *v, double *g, double *diag, double *Hv)
{
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    if (g) memset(g, 0, sizeof(double) * 3 * nnodes);
    if (diag) memset(diag, 0, sizeof(double) * 3 * nnodes);
    if (Hv) memset(Hv, 0, sizeof(double) * 3 * nnodes);
    double K = 0.0;
    for (int64_t i = 0; i < npts; ++i) {
        int64_t node[8];
        double w[8];
        if (!kp_weights(nn, H, x + 3 * i, node, w)) return NAN;
        double res[3], pv[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
            double yu = x[3 * i + a];
            for (int q = 0; q < 8; ++q) yu += w[q] * u[a * nnodes + node[q]];
            res[a] = yu - tgt[3 * i + a];
            K += res[a] * res[a];
            if (v)
                for (int q = 0; q < 8; ++q) pv[a] += w[q] * v[a * nnodes + node[q]];
        }
        for (int q = 0; q < 8; ++q)
            for (int a = 0; a < 3; ++a) {
                if (g) g[a * nnodes + node[q]] += 2.0 * w[q] * res[a];
                if (diag) diag[a * nnodes + node[q]] += 2.0 * w[q] * w[q];
                if (Hv) Hv[a * nnodes + node[q]] += 2.0 * w[q] * pv[a];
            }
    }
    return K;
}

/* ------------------------------------------------------------------------------ */
/* Exact determinant of grad y at every voxel centre (diagnostic only).             */
/* ------------------------------------------------------------------------------ */
void or_det_voxels(const int64_t *n, const int64_t *m, const double *h, const double *u, double *det)
{
    int64_t nn[3];
    node_counts(n, m, nn);
    double H[3] = {h[0] * m[0], h[1] * m[1], h[2] * m[2]};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n[2]; ++k)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                int64_t cell[3];
                double xi[3];
                axis_weights(i, m[0], &cell[0], &xi[0]);
                axis_weights(j, m[1], &cell[1], &xi[1]);
                axis_weights(k, m[2], &cell[2], &xi[2]);
                double alpha[64], d[64], de;
                or_vcc_cell_expansion(nn, H, u, cell, xi, alpha, d, &de);
                det[IDX3(i, j, k, n[0], n[1])] = de;
            }
}

/* number of threads the parallel loops use (for reporting) */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the number of threads of the parallel loops (n >= 1; for timing runs) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------ */
/* Derivative of the NGF distance (eq. 1) with respect to the moving image values.   */
/* D depends on T only through a_v = G(y_v), the trilinear sample of grad T, so       */
/*   dD/d(grad T)[p] = sum_v w_{v,p} (-2 h^3 r_v dr/da_v)   (w: trilinear weights),   */
/* and grad T is the central-difference stencil of T with replicated borders, so     */
/*   dD/dT = stencil^T (dD/d grad T).                                                 */
/* Output dT is [N] (same layout as T).                                              */
/* ------------------------------------------------------------------------------ */
void or_ngf_grad_T(const int64_t *n, const double *h, const int64_t *m, double eta, const double *gR,
                   const double *gT, const double *u, double *dT)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const double h3 = h[0] * h[1] * h[2];
    const double e2 = eta * eta;
    double *wv = (double *)malloc(sizeof(double) * 3 * nvox); /* -2 h^3 r dr/da per voxel */
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * 3 * nvox);
    double *tt = (double *)malloc(sizeof(double) * 3 * nvox);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t v = IDX3(i, j, k, nx, ny);
                const int64_t idx[3] = {i, j, k};
                double uh[3], t[3], a[3], JG[3][3];
                int64_t i0[3];
                voxel_uh(nn, m, h, u, i, j, k, uh);
                for (int q = 0; q < 3; ++q) split_axis(idx[q], uh[q], n[q], &i0[q], &t[q]);
                sample_vec_at(n, h, gT, i0, t, a, JG);
                const double *b = gR + 3 * v;
                double Da = e2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                double Db = e2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                double P = e2 + a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
                double sq = sqrt(Da * Db);
                double r = P / sq;
                for (int q = 0; q < 3; ++q) {
                    wv[3 * v + q] = -2.0 * h3 * r * (b[q] - (P / Da) * a[q]) / sq;
                    cell[3 * v + q] = i0[q];
                    tt[3 * v + q] = t[q];
                }
            }
    /* scatter onto the grad-T grid with the trilinear weights (zero outside) */
    double *W = (double *)calloc((size_t)(3 * nvox), sizeof(double));
    for (int64_t v = 0; v < nvox; ++v) {
        const double *t = tt + 3 * v;
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    int64_t ii = cell[3 * v] + cx, jj = cell[3 * v + 1] + cy, kk = cell[3 * v + 2] + cz;
                    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
                    double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
                    for (int c = 0; c < 3; ++c) W[3 * IDX3(ii, jj, kk, nx, ny) + c] += w * wv[3 * v + c];
                }
    }
    /* transpose of (grad I)_a[i] = (I[clamp(i+e_a)] - I[clamp(i-e_a)]) / (2 h_a) */
    memset(dT, 0, sizeof(double) * nvox);
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t v = IDX3(i, j, k, nx, ny);
                int64_t ip = i < nx - 1 ? i + 1 : nx - 1, im = i > 0 ? i - 1 : 0;
                int64_t jp = j < ny - 1 ? j + 1 : ny - 1, jm = j > 0 ? j - 1 : 0;
                int64_t kp = k < nz - 1 ? k + 1 : nz - 1, km = k > 0 ? k - 1 : 0;
                dT[IDX3(ip, j, k, nx, ny)] += W[3 * v] / (2.0 * h[0]);
                dT[IDX3(im, j, k, nx, ny)] -= W[3 * v] / (2.0 * h[0]);
                dT[IDX3(i, jp, k, nx, ny)] += W[3 * v + 1] / (2.0 * h[1]);
                dT[IDX3(i, jm, k, nx, ny)] -= W[3 * v + 1] / (2.0 * h[1]);
                dT[IDX3(i, j, kp, nx, ny)] += W[3 * v + 2] / (2.0 * h[2]);
                dT[IDX3(i, j, km, nx, ny)] -= W[3 * v + 2] / (2.0 * h[2]);
            }
    free(W);
    free(wv);
    free(cell);
    free(tt);
}

/* ------------------------------------------------------------------------------ */
/* Lung-boundary term, eq. 6: B = 1/2 int (b_M(y(x)) - b_F(x))^2 dx with the binary  */
/* masks b_F (fixed, at the voxel centres) and b_M (moving, sampled at y(x_v) by      */
/* trilinear interpolation with zero outside the volume, like grad T in eq. 1):      */
/*   res_v = b_M(y_v) - b_F(x_v),   B = 1/2 h^3 sum_v res_v^2.                        */
/* With sb_v = grad b_M(y_v) (the gradient of the trilinear interpolant in mm, in    */
/* the cell floor(q), one-sided on a face like JG in eq. 1):                          */
/*   grad B = h^3 sum_v phi_v res_v sb_v,                                             */
/*   Gauss-Newton matrix h^3 J^T J with J_v = phi_v sb_v^T (exact form of the SSD     */
/*   Gauss-Newton matrix), diagonal h^3 sum_v phi_v^2 sb_v^2.                          */
/* bF, bM are [N] volumes; u a node field; g, diag, sb ([N][3]), res ([N]) optional.  */
/* Returns B.                                                                          */
/* ------------------------------------------------------------------------------ */
static void sample_scalar_at(const int64_t *n, const double *h, const double *f, const int64_t i0[3],
                             const double t[3], double *val, double grad[3])
{
    *val = 0.0;
    grad[0] = grad[1] = grad[2] = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                int64_t ii = i0[0] + cx, jj = i0[1] + cy, kk = i0[2] + cz;
                if (ii < 0 || ii >= n[0] || jj < 0 || jj >= n[1] || kk < 0 || kk >= n[2]) continue;
                const double fv = f[IDX3(ii, jj, kk, n[0], n[1])];
                double wx = cx ? t[0] : 1.0 - t[0], dwx = cx ? 1.0 : -1.0;
                double wy = cy ? t[1] : 1.0 - t[1], dwy = cy ? 1.0 : -1.0;
                double wz = cz ? t[2] : 1.0 - t[2], dwz = cz ? 1.0 : -1.0;
                *val += wx * wy * wz * fv;
                grad[0] += dwx * wy * wz * fv / h[0];
                grad[1] += wx * dwy * wz * fv / h[1];
                grad[2] += wx * wy * dwz * fv / h[2];
            }
}

double or_mask(const int64_t *n, const double *h, const int64_t *m, const double *bF, const double *bM,
               const double *u, double *g, double *diag, double *sb_out, double *res_out)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double h3 = h[0] * h[1] * h[2];
    double *res = (double *)malloc(sizeof(double) * nvox);
    double *sb = (double *)malloc(sizeof(double) * 3 * nvox);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t v = IDX3(i, j, k, nx, ny);
                const int64_t idx[3] = {i, j, k};
                double uh[3], t[3], val;
                int64_t i0[3];
                voxel_uh(nn, m, h, u, i, j, k, uh);
                for (int q = 0; q < 3; ++q) split_axis(idx[q], uh[q], n[q], &i0[q], &t[q]);
                sample_scalar_at(n, h, bM, i0, t, &val, sb + 3 * v);
                res[v] = val - bF[v];
            }
    double B = 0.0;
    for (int64_t v = 0; v < nvox; ++v) B += res[v] * res[v];
    B *= 0.5 * h3;
    if (g) memset(g, 0, sizeof(double) * 3 * nnodes);
    if (diag) memset(diag, 0, sizeof(double) * 3 * nnodes);
    if (g || diag) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t v = IDX3(i, j, k, nx, ny);
                    double val[3];
                    if (g) {
                        for (int t = 0; t < 3; ++t) val[t] = h3 * res[v] * sb[3 * v + t];
                        scatter_voxel(nn, m, g, i, j, k, val, 0);
                    }
                    if (diag) {
                        for (int t = 0; t < 3; ++t) val[t] = h3 * sb[3 * v + t] * sb[3 * v + t];
                        scatter_voxel(nn, m, diag, i, j, k, val, 1);
                    }
                }
    }
    if (sb_out) memcpy(sb_out, sb, sizeof(double) * 3 * nvox);
    if (res_out) memcpy(res_out, res, sizeof(double) * nvox);
    free(res);
    free(sb);
    return B;
}

/* Sample-cell ties of the lung-boundary term (see or_ngf_ties for the tie rule): the  */
/* sampled mask value is continuous across a face, its gradient sb is one-sided.  Per  */
/* node: ag = sum_v phi_v max |h^3 res (sb'_c - sb_c)|, adg = sum_v phi_v^2             */
/* max |h^3 (sb'_c^2 - sb_c^2)|, ahv = sum_v phi_v max |h^3 (sb'_c (sb'.w) - sb_c       */
/* (sb.w))| with w = (Pv)(x_v); per voxel sbdev = max |sb'_c - sb_c|.  Returns the     */
/* number of voxels with a tie.                                                       */
int64_t or_mask_ties(const int64_t *n, const double *h, const int64_t *m, const double *bF, const double *bM,
                     const double *u, const double *v, double *ag, double *adg, double *ahv, double *sbdev)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    const int64_t nvox = nx * ny * nz;
    int64_t nn[3];
    node_counts(n, m, nn);
    const int64_t nnodes = nn[0] * nn[1] * nn[2];
    const double h3 = h[0] * h[1] * h[2];
    if (ag) memset(ag, 0, sizeof(double) * 3 * nnodes);
    if (adg) memset(adg, 0, sizeof(double) * 3 * nnodes);
    if (ahv) memset(ahv, 0, sizeof(double) * 3 * nnodes);
    if (sbdev) memset(sbdev, 0, sizeof(double) * 3 * nvox);
    int64_t nt = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t vox = IDX3(i, j, k, nx, ny);
                const int64_t idx[3] = {i, j, k};
                double uh[3], t0[3], at[3], w[3] = {0.0, 0.0, 0.0};
                int64_t i00[3], ai[3];
                voxel_uh(nn, m, h, u, i, j, k, uh);
                const int mask = tie_axes(nn, m, n, h, u, i, j, k, uh, ai, at);
                if (!mask) continue;
                ++nt;
                for (int a = 0; a < 3; ++a) split_axis(idx[a], uh[a], n[a], &i00[a], &t0[a]);
                if (v) interp_voxel(nn, m, v, i, j, k, w);
                double val0, sb0[3];
                sample_scalar_at(n, h, bM, i00, t0, &val0, sb0);
                const double res = val0 - bF[vox];
                const double sw0 = sb0[0] * w[0] + sb0[1] * w[1] + sb0[2] * w[2];
                double o[12] = {0.0};
                for (int combo = 1; combo < 8; ++combo) {
                    if (combo & ~mask) continue;
                    int64_t i1[3];
                    double t1[3], val1, sb1[3];
                    for (int a = 0; a < 3; ++a) {
                        i1[a] = (combo >> a & 1) ? ai[a] : i00[a];
                        t1[a] = (combo >> a & 1) ? at[a] : t0[a];
                    }
                    sample_scalar_at(n, h, bM, i1, t1, &val1, sb1);
                    const double sw1 = sb1[0] * w[0] + sb1[1] * w[1] + sb1[2] * w[2];
                    for (int q = 0; q < 3; ++q) {
                        const double dg = fabs(h3 * res * (sb1[q] - sb0[q]));
                        const double dd = fabs(h3 * (sb1[q] * sb1[q] - sb0[q] * sb0[q]));
                        const double dh = fabs(h3 * (sb1[q] * sw1 - sb0[q] * sw0));
                        const double ds = fabs(sb1[q] - sb0[q]);
                        if (dg > o[q]) o[q] = dg;
                        if (dd > o[3 + q]) o[3 + q] = dd;
                        if (dh > o[6 + q]) o[6 + q] = dh;
                        if (ds > o[9 + q]) o[9 + q] = ds;
                    }
                }
                if (ag) scatter_voxel(nn, m, ag, i, j, k, o, 0);
                if (adg) scatter_voxel(nn, m, adg, i, j, k, o + 3, 1);
                if (ahv) scatter_voxel(nn, m, ahv, i, j, k, o + 6, 0);
                if (sbdev)
                    for (int q = 0; q < 3; ++q) sbdev[3 * vox + q] = o[9 + q];
            }
    return nt;
}

/* ------------------------------------------------------------------------------ */
/* Keypoint matching cost, eq. 2 (Sec. II-C2), on images at isotropic resolution:   */
/*   D_KP(k, d) = 1/|P| sum_{p in P_k} [1 - <grad M(p+d), grad F(p)>_eta^2 /         */
/*                                    (|grad M(p+d)|_eta^2 |grad F(p)|_eta^2)]        */
/* with <f,g>_eta = eta^2 + f.g as in eq. 1 (cancellation-free form of 1 - r^2).     */
/* Keypoints k are voxel indices; P_k = k + {-3,-1,1,3}^3 (a 7^3 patch, stride 2,    */
/* 64 voxels); labels d = step (i - R) voxels per axis, i = 0..2R, ordered           */
/* [iz][iy][ix].  Gradients outside the volume are zero (zero padding).              */
/* gF, gM: [N][3] gradient images.  out: [nkp][(2R+1)^3].                             */
/* ------------------------------------------------------------------------------ */
void or_kp_cost(const int64_t *n, const double *gF, const double *gM, int64_t nkp, const int64_t *kp,
                double eta, int64_t R, int64_t step, double *out)
{
    const int64_t nl = 2 * R + 1, L = nl * nl * nl;
    const double e2 = eta * eta;
    static const int off[4] = {-3, -1, 1, 3};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nkp * nl; ++q) {
        const int64_t k = q / nl, iz = q % nl;
        const int64_t *kv = kp + 3 * k;
        for (int64_t iy = 0; iy < nl; ++iy)
            for (int64_t ix = 0; ix < nl; ++ix) {
                const int64_t d[3] = {step * (ix - R), step * (iy - R), step * (iz - R)};
                double sum = 0.0;
                for (int oz = 0; oz < 4; ++oz)
                    for (int oy = 0; oy < 4; ++oy)
                        for (int ox = 0; ox < 4; ++ox) {
                            const int64_t p[3] = {kv[0] + off[ox], kv[1] + off[oy], kv[2] + off[oz]};
                            double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
                            const int64_t pd[3] = {p[0] + d[0], p[1] + d[1], p[2] + d[2]};
                            if (p[0] >= 0 && p[0] < n[0] && p[1] >= 0 && p[1] < n[1] && p[2] >= 0 && p[2] < n[2]) {
                                const double *g = gF + 3 * IDX3(p[0], p[1], p[2], n[0], n[1]);
                                b[0] = g[0]; b[1] = g[1]; b[2] = g[2];
                            }
                            if (pd[0] >= 0 && pd[0] < n[0] && pd[1] >= 0 && pd[1] < n[1] && pd[2] >= 0 && pd[2] < n[2]) {
                                const double *g = gM + 3 * IDX3(pd[0], pd[1], pd[2], n[0], n[1]);
                                a[0] = g[0]; a[1] = g[1]; a[2] = g[2];
                            }
                            const double Da = e2 + a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
                            const double Db = e2 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                            const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
                            const double cx = a[1] * b[2] - a[2] * b[1];
                            const double cy = a[2] * b[0] - a[0] * b[2];
                            const double cz = a[0] * b[1] - a[1] * b[0];
                            sum += (e2 * (dx * dx + dy * dy + dz * dz) + cx * cx + cy * cy + cz * cz) / (Da * Db);
                        }
                out[k * L + (iz * nl + iy) * nl + ix] = sum / 64.0;
            }
    }
}
