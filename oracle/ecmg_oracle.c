/*
 * CPU FP64 oracle for the ECMG_jcg cascade (Pan, He & Hu, "A new extrapolation
 * cascadic multigrid method for 3D elliptic boundary value problems on
 * rectangular domains", arXiv 1506.02983).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or calls
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   - Q1 element matrices are integrated numerically (2x2x2 Gauss), not taken
 *     from a closed form (Section 2, eqs. var and fe_equation);
 *   - the global matrix is assembled into CSR;
 *   - the two coarsest grids are solved directly (banded Cholesky, DSOLVE of
 *     Algorithm 4);
 *   - JCG is textbook preconditioned CG with M = diag(A) (Section 4.1);
 *   - EXP_finite and EXP_true evaluate the paper's formulas node by node
 *     (Sections 4.2-4.3, eqs. jiedian, zhongdian, inter, t1, chenlin).
 * Dot products are plain sequential FP64 sums in node-index order.  OpenMP is
 * used only for loops whose result does not depend on the thread count
 * (row-parallel matrix-vector products, assembly by rows, pointwise updates).
 *
 * Grid conventions: level with nx x ny x nz elements; node (i,j,k) has index
 * i + (nx+1)*(j + (ny+1)*k) (x fastest), element (i,j,k) index i + nx*(j + ny*k).
 * Faces are numbered 0..5 = x-lo, x-hi, y-lo, y-hi, z-lo, z-hi.  Face type 0 is
 * Dirichlet, 1 is Robin (Neumann = Robin with alpha = 0, Section 1).
 * A node on any Dirichlet face is a Dirichlet node.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t nx, ny, nz;      /* elements per axis */
    double hx, hy, hz;       /* element sides */
    int32_t face_type[6];    /* 0 = Dirichlet, 1 = Robin */
} orc_grid;

typedef struct {
    int64_t n;               /* rows (all nodes) */
    int64_t nnz;
    int64_t *rowptr;         /* n+1 */
    int32_t *col;            /* nnz */
    double *val;             /* nnz */
} orc_csr;

/* 1/sqrt(3): the abscissa of 2-point Gauss-Legendre quadrature on [-1,1]. */
#define ORC_GAUSS 0.57735026918962576450914878050196

static inline int64_t nid(const orc_grid *g, int64_t i, int64_t j, int64_t k) {
    return i + (g->nx + 1) * (j + (g->ny + 1) * k);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following parallel regions (n >= 1); timing only */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Node (i,j,k) lies on a Dirichlet face (Dirichlet wins on shared edges). */
static int is_dirichlet(const orc_grid *g, int64_t i, int64_t j, int64_t k) {
    const int32_t *t = g->face_type;
    return (i == 0 && t[0] == 0) || (i == g->nx && t[1] == 0) ||
           (j == 0 && t[2] == 0) || (j == g->ny && t[3] == 0) ||
           (k == 0 && t[4] == 0) || (k == g->nz && t[5] == 0);
}

void orc_dirichlet_mask(const orc_grid *g, uint8_t *mask) {
    #pragma omp parallel for
    for (int64_t k = 0; k <= g->nz; k++)
        for (int64_t j = 0; j <= g->ny; j++)
            for (int64_t i = 0; i <= g->nx; i++)
                mask[nid(g, i, j, k)] = (uint8_t)is_dirichlet(g, i, j, k);
}

/* ------------------------------------------------------------------------ */
/* Element matrices (Section 2: a(u,v) = int beta grad u.grad v + int_R alpha u v) */
/* ------------------------------------------------------------------------ */

/* Q1 stiffness of one hexahedron of sides hx,hy,hz with beta = 1:
 * K[a*8+b] = int_e grad phi_a . grad phi_b, by 2x2x2 Gauss (exact for Q1).
 * Local node a = ax + 2 ay + 4 az with natural coordinates (2ax-1, 2ay-1, 2az-1). */
void orc_element_stiffness(double hx, double hy, double hz, double *K) {
    memset(K, 0, 64 * sizeof(double));
    const double w = hx * hy * hz / 8.0;  /* |J| for [-1,1]^3 -> element, unit weights */
    for (int gz = 0; gz < 2; gz++)
    for (int gy = 0; gy < 2; gy++)
    for (int gx = 0; gx < 2; gx++) {
        const double s = gx ? ORC_GAUSS : -ORC_GAUSS;
        const double t = gy ? ORC_GAUSS : -ORC_GAUSS;
        const double u = gz ? ORC_GAUSS : -ORC_GAUSS;
        double grad[8][3];
        for (int a = 0; a < 8; a++) {
            const double xa = 2.0 * (a & 1) - 1.0;
            const double ya = 2.0 * ((a >> 1) & 1) - 1.0;
            const double za = 2.0 * ((a >> 2) & 1) - 1.0;
            /* phi_a = (1+xa s)(1+ya t)(1+za u)/8; d/dx = (2/hx) d/ds */
            grad[a][0] = (2.0 / hx) * 0.125 * xa * (1.0 + ya * t) * (1.0 + za * u);
            grad[a][1] = (2.0 / hy) * 0.125 * (1.0 + xa * s) * ya * (1.0 + za * u);
            grad[a][2] = (2.0 / hz) * 0.125 * (1.0 + xa * s) * (1.0 + ya * t) * za;
        }
        for (int a = 0; a < 8; a++)
            for (int b = 0; b < 8; b++)
                K[a * 8 + b] += w * (grad[a][0] * grad[b][0] + grad[a][1] * grad[b][1] +
                                     grad[a][2] * grad[b][2]);
    }
}

/* Q1 mass matrix of one rectangular face element of sides hp,hq:
 * M[a*4+b] = int_f phi_a phi_b by 2x2 Gauss (exact), local node a = ap + 2 aq. */
void orc_face_mass(double hp, double hq, double *M) {
    memset(M, 0, 16 * sizeof(double));
    const double w = hp * hq / 4.0;
    for (int gq = 0; gq < 2; gq++)
    for (int gp = 0; gp < 2; gp++) {
        const double s = gp ? ORC_GAUSS : -ORC_GAUSS;
        const double t = gq ? ORC_GAUSS : -ORC_GAUSS;
        double phi[4];
        for (int a = 0; a < 4; a++) {
            const double pa = 2.0 * (a & 1) - 1.0, qa = 2.0 * ((a >> 1) & 1) - 1.0;
            phi[a] = 0.25 * (1.0 + pa * s) * (1.0 + qa * t);
        }
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) M[a * 4 + b] += w * phi[a] * phi[b];
    }
}

/* Geometry of face f: the in-face axes (p,q), the normal axis, the node index
 * along the normal, and the face-element counts. */
static void face_axes(const orc_grid *g, int f, int *pax, int *qax, int *nax, int64_t *nfix,
                      int64_t *np, int64_t *nq, double *hp, double *hq) {
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    const double h[3] = {g->hx, g->hy, g->hz};
    const int ax = f / 2;
    int p = (ax == 0) ? 1 : 0;
    int q = (ax == 2) ? 1 : 2;
    *pax = p; *qax = q; *nax = ax;
    *nfix = (f % 2 == 0) ? 0 : n[ax];
    *np = n[p]; *nq = n[q]; *hp = h[p]; *hq = h[q];
}

/* ------------------------------------------------------------------------ */
/* Assembly: A = sum_e beta_e K_e + sum_f alpha_f M_f, stored as CSR over all  */
/* nodes with every in-grid 27-point neighbour as a structural entry.          */
/* beta: element array; alpha[f]: face-element array of face f (p fastest),   */
/* NULL for Dirichlet faces.                                                   */
/* ------------------------------------------------------------------------ */

int64_t orc_csr_nnz(const orc_grid *g) {
    /* count of in-grid offsets per axis summed over nodes = product of sums */
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    int64_t prod = 1;
    for (int d = 0; d < 3; d++) {
        const int64_t m = n[d] + 1;
        /* sum over positions of the number of valid offsets in {-1,0,1} */
        const int64_t s = (m == 1) ? 1 : 3 * m - 2;
        prod *= s;
    }
    return prod;
}

int orc_assemble(const orc_grid *g, const double *beta, const double *const *alpha,
                 int64_t *rowptr, int32_t *col, double *val) {
    double K[64];
    orc_element_stiffness(g->hx, g->hy, g->hz, K);
    const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    const int64_t n = (nx + 1) * (ny + 1) * (nz + 1);

    /* row pointers: rows in index order, columns in increasing index order */
    rowptr[0] = 0;
    for (int64_t k = 0; k <= nz; k++)
        for (int64_t j = 0; j <= ny; j++)
            for (int64_t i = 0; i <= nx; i++) {
                const int64_t cx = (i > 0) + 1 + (i < nx);
                const int64_t cy = (j > 0) + 1 + (j < ny);
                const int64_t cz = (k > 0) + 1 + (k < nz);
                const int64_t r = nid(g, i, j, k);
                rowptr[r + 1] = rowptr[r] + cx * cy * cz;
            }
    (void)n;

    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k <= nz; k++) {
        double M[16];
        for (int64_t j = 0; j <= ny; j++)
            for (int64_t i = 0; i <= nx; i++) {
                double row[27];
                memset(row, 0, sizeof(row));
                /* stiffness: every element containing node (i,j,k) */
                for (int64_t ke = k - 1; ke <= k; ke++) {
                    if (ke < 0 || ke >= nz) continue;
                    for (int64_t je = j - 1; je <= j; je++) {
                        if (je < 0 || je >= ny) continue;
                        for (int64_t ie = i - 1; ie <= i; ie++) {
                            if (ie < 0 || ie >= nx) continue;
                            const double b = beta[ie + nx * (je + ny * ke)];
                            const int a = (int)((i - ie) + 2 * (j - je) + 4 * (k - ke));
                            for (int c = 0; c < 8; c++) {
                                const int64_t ci = ie + (c & 1), cj = je + ((c >> 1) & 1),
                                              ck = ke + ((c >> 2) & 1);
                                const int slot = (int)((ci - i + 1) + 3 * (cj - j + 1) + 9 * (ck - k + 1));
                                row[slot] += b * K[a * 8 + c];
                            }
                        }
                    }
                }
                /* Robin faces through this node */
                for (int f = 0; f < 6; f++) {
                    if (g->face_type[f] != 1 || alpha == NULL || alpha[f] == NULL) continue;
                    int pax, qax, nax; int64_t nfix, np, nq; double hp, hq;
                    face_axes(g, f, &pax, &qax, &nax, &nfix, &np, &nq, &hp, &hq);
                    const int64_t idx[3] = {i, j, k};
                    if (idx[nax] != nfix) continue;
                    orc_face_mass(hp, hq, M);
                    const int64_t pi = idx[pax], qi = idx[qax];
                    for (int64_t eq = qi - 1; eq <= qi; eq++) {
                        if (eq < 0 || eq >= nq) continue;
                        for (int64_t ep = pi - 1; ep <= pi; ep++) {
                            if (ep < 0 || ep >= np) continue;
                            const double al = alpha[f][ep + np * eq];
                            const int a = (int)((pi - ep) + 2 * (qi - eq));
                            for (int c = 0; c < 4; c++) {
                                int64_t cidx[3] = {i, j, k};
                                cidx[pax] = ep + (c & 1);
                                cidx[qax] = eq + ((c >> 1) & 1);
                                const int slot = (int)((cidx[0] - i + 1) + 3 * (cidx[1] - j + 1) +
                                                       9 * (cidx[2] - k + 1));
                                row[slot] += al * M[a * 4 + c];
                            }
                        }
                    }
                }
                /* compress the in-grid slots */
                const int64_t r = nid(g, i, j, k);
                int64_t pos = rowptr[r];
                for (int s = 0; s < 27; s++) {
                    const int64_t di = s % 3 - 1, dj = (s / 3) % 3 - 1, dk = s / 9 - 1;
                    const int64_t ci = i + di, cj = j + dj, ck = k + dk;
                    if (ci < 0 || ci > nx || cj < 0 || cj > ny || ck < 0 || ck > nz) continue;
                    col[pos] = (int32_t)nid(g, ci, cj, ck);
                    val[pos] = row[s];
                    pos++;
                }
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Load vector f(v) = int f v + int_R g_R v (Section 2), 2x2x2 Gauss per     */
/* element and 2x2 Gauss per Robin face element.                             */
/* fg: f at the Gauss points, array (2nz) x (2ny) x (2nx), x fastest, where   */
/* element e's points along an axis are e's origin + (1 -/+ 1/sqrt3) h/2.     */
/* gR[f]: g_R at face f's Gauss points, (2nq) x (2np), p fastest; NULL if not */
/* Robin.                                                                     */
/* ------------------------------------------------------------------------ */
int orc_load(const orc_grid *g, const double *fg, const double *const *gR, double *F) {
    const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    const double w = g->hx * g->hy * g->hz / 8.0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k <= nz; k++)
        for (int64_t j = 0; j <= ny; j++)
            for (int64_t i = 0; i <= nx; i++) {
                double s = 0.0;
                for (int64_t ke = k - 1; ke <= k; ke++) {
                    if (ke < 0 || ke >= nz) continue;
                    for (int64_t je = j - 1; je <= j; je++) {
                        if (je < 0 || je >= ny) continue;
                        for (int64_t ie = i - 1; ie <= i; ie++) {
                            if (ie < 0 || ie >= nx) continue;
                            const double xa = 2.0 * (double)(i - ie) - 1.0;
                            const double ya = 2.0 * (double)(j - je) - 1.0;
                            const double za = 2.0 * (double)(k - ke) - 1.0;
                            for (int gz = 0; gz < 2; gz++)
                            for (int gy = 0; gy < 2; gy++)
                            for (int gx = 0; gx < 2; gx++) {
                                const double ss = gx ? ORC_GAUSS : -ORC_GAUSS;
                                const double tt = gy ? ORC_GAUSS : -ORC_GAUSS;
                                const double uu = gz ? ORC_GAUSS : -ORC_GAUSS;
                                const double phi = 0.125 * (1.0 + xa * ss) * (1.0 + ya * tt) * (1.0 + za * uu);
                                const double fv = fg[(2 * ke + gz) * (2 * ny) * (2 * nx) +
                                                     (2 * je + gy) * (2 * nx) + (2 * ie + gx)];
                                s += w * fv * phi;
                            }
                        }
                    }
                }
                for (int f = 0; f < 6; f++) {
                    if (g->face_type[f] != 1 || gR == NULL || gR[f] == NULL) continue;
                    int pax, qax, nax; int64_t nfix, np, nq; double hp, hq;
                    face_axes(g, f, &pax, &qax, &nax, &nfix, &np, &nq, &hp, &hq);
                    const int64_t idx[3] = {i, j, k};
                    if (idx[nax] != nfix) continue;
                    const double wf = hp * hq / 4.0;
                    const int64_t pi = idx[pax], qi = idx[qax];
                    for (int64_t eq = qi - 1; eq <= qi; eq++) {
                        if (eq < 0 || eq >= nq) continue;
                        for (int64_t ep = pi - 1; ep <= pi; ep++) {
                            if (ep < 0 || ep >= np) continue;
                            const double pa = 2.0 * (double)(pi - ep) - 1.0;
                            const double qa = 2.0 * (double)(qi - eq) - 1.0;
                            for (int gq = 0; gq < 2; gq++)
                            for (int gp = 0; gp < 2; gp++) {
                                const double ss = gp ? ORC_GAUSS : -ORC_GAUSS;
                                const double tt = gq ? ORC_GAUSS : -ORC_GAUSS;
                                const double phi = 0.25 * (1.0 + pa * ss) * (1.0 + qa * tt);
                                s += wf * gR[f][(2 * eq + gq) * (2 * np) + (2 * ep + gp)] * phi;
                            }
                        }
                    }
                }
                F[nid(g, i, j, k)] = s;
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Linear algebra on the free unknowns                                        */
/* ------------------------------------------------------------------------ */

/* y = A v restricted to free rows; Dirichlet rows of y are 0.  All columns are
 * used, so with v = g_D on Dirichlet nodes this is A_FF v_F + A_FD g_D. */
void orc_spmv(const orc_csr *A, const uint8_t *dmask, const double *v, double *y) {
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n; r++) {
        if (dmask[r]) { y[r] = 0.0; continue; }
        double s = 0.0;
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; p++) s += A->val[p] * v[A->col[p]];
        y[r] = s;
    }
}

/* Plain sequential dot product in index order. */
static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* Diagonal of A on free rows (the Jacobi preconditioner M = diag(A_FF)). */
void orc_diagonal(const orc_csr *A, double *D) {
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n; r++) {
        double d = 0.0;
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; p++)
            if (A->col[p] == r) d = A->val[p];
        D[r] = d;
    }
}

/* b = F - A_FD g_D on free rows (Dirichlet lifting), 0 on Dirichlet rows.
 * gD: node array; only Dirichlet entries are used. Returns ||b||_2 (free rows). */
double orc_lift(const orc_csr *A, const uint8_t *dmask, const double *F, const double *gD, double *b) {
    const int64_t n = A->n;
    double *t = (double *)malloc((size_t)n * sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; r++) t[r] = dmask[r] ? gD[r] : 0.0;
    orc_spmv(A, dmask, t, b);
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; r++) b[r] = dmask[r] ? 0.0 : F[r] - b[r];
    free(t);
    return sqrt(dot(n, b, b));
}

/* ||f_h||_2 of the stopping test of Algorithm 4: the right-hand side of the
 * system A_h u_h = f_h in which every Dirichlet node keeps an identity row,
 * i.e. f_h = b on free nodes and g_D on Dirichlet nodes, summed in index order. */
double orc_rhs_norm(int64_t n, const uint8_t *dmask, const double *b, const double *gD) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double v = dmask[i] ? gD[i] : b[i];
        s += v * v;
    }
    return sqrt(s);
}

/* JCG (Algorithm 4 with the Jacobi-preconditioned CG of Section 4.1).
 * x: in = initial guess with g_D on Dirichlet nodes; out = final iterate.
 * The loop runs while ||r||_2 > eps nf (checked before the first step, the
 * `while` of Algorithm 4) and k < max_iter, where nf = ||f_h||_2 from
 * orc_rhs_norm (r vanishes on Dirichlet rows); with fixed_iters >= 0 it runs
 * exactly fixed_iters steps instead.  hist (optional, length max(max_iter,
 * fixed_iters)+1) receives ||r_k||_2.
 * Returns 0, -3 (max_iter reached without convergence) or -4 (breakdown). */
int orc_jcg(const orc_csr *A, const uint8_t *dmask, const double *D, const double *F,
            double *x, double eps, int64_t max_iter, int64_t fixed_iters, double nf,
            int64_t *iters_out, double *rre_out, double *rre_true_out, double *hist) {
    const int64_t n = A->n;
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *z = (double *)calloc((size_t)n, sizeof(double));
    double *p = (double *)calloc((size_t)n, sizeof(double));
    double *q = (double *)calloc((size_t)n, sizeof(double));
    int status = 0;

    orc_spmv(A, dmask, x, q);                       /* r = F - A x on free rows */
    for (int64_t i = 0; i < n; i++) r[i] = dmask[i] ? 0.0 : F[i] - q[i];
    double rn = sqrt(dot(n, r, r));
    if (hist) hist[0] = rn;
    double rho = 0.0;
    int64_t k = 0;
    for (;;) {
        if (fixed_iters >= 0) {
            if (k >= fixed_iters) break;
        } else {
            if (!(rn > eps * nf)) break;
            if (k >= max_iter) { status = -3; break; }
        }
        for (int64_t i = 0; i < n; i++) z[i] = dmask[i] ? 0.0 : r[i] / D[i];
        const double rho_new = dot(n, r, z);
        if (k == 0) {
            for (int64_t i = 0; i < n; i++) p[i] = z[i];
        } else {
            const double bet = rho_new / rho;
            for (int64_t i = 0; i < n; i++) p[i] = z[i] + bet * p[i];
        }
        rho = rho_new;
        orc_spmv(A, dmask, p, q);
        const double pq = dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = -4; break; }
        const double alpha = rho / pq;
        for (int64_t i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        k++;
        rn = sqrt(dot(n, r, r));
        if (hist) hist[k] = rn;
    }
    *iters_out = k;
    *rre_out = (nf > 0.0) ? rn / nf : 0.0;
    /* true residual */
    orc_spmv(A, dmask, x, q);
    for (int64_t i = 0; i < n; i++) q[i] = dmask[i] ? 0.0 : F[i] - q[i];
    *rre_true_out = (nf > 0.0) ? sqrt(dot(n, q, q)) / nf : 0.0;
    free(r); free(z); free(p); free(q);
    return status;
}

/* DSOLVE (Algorithm 4, the two coarsest grids): exact solve of
 * A_FF x_F = F_F - A_FD g_D by banded Cholesky.  The free unknowns are ordered
 * lexicographically with the axis of fewest nodes fastest, which keeps the
 * band narrow.  x: in = g_D on Dirichlet nodes; out = solution. */
int orc_dsolve(const orc_grid *g, const orc_csr *A, const uint8_t *dmask, const double *F, double *x) {
    const int64_t n = A->n;
    const int64_t m[3] = {g->nx + 1, g->ny + 1, g->nz + 1};
    int order[3] = {0, 1, 2};               /* order[0] = fastest axis */
    for (int a = 0; a < 3; a++)
        for (int b = a + 1; b < 3; b++)
            if (m[order[b]] < m[order[a]]) { int t = order[a]; order[a] = order[b]; order[b] = t; }

    int64_t *perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));   /* node -> unknown or -1 */
    int64_t *node_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t nf = 0;
    int64_t c[3];
    for (c[2] = 0; c[2] < m[order[2]]; c[2]++)
        for (c[1] = 0; c[1] < m[order[1]]; c[1]++)
            for (c[0] = 0; c[0] < m[order[0]]; c[0]++) {
                int64_t ijk[3];
                ijk[order[0]] = c[0]; ijk[order[1]] = c[1]; ijk[order[2]] = c[2];
                const int64_t r = nid(g, ijk[0], ijk[1], ijk[2]);
                if (dmask[r]) { perm[r] = -1; continue; }
                perm[r] = nf; node_of[nf] = r; nf++;
            }
    /* right-hand side b = F - A_FD g_D, and the half bandwidth */
    double *rhs = (double *)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(double));
    int64_t bw = 0;
    for (int64_t u = 0; u < nf; u++) {
        const int64_t r = node_of[u];
        double s = F[r];
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; p++) {
            const int64_t cc = A->col[p];
            if (dmask[cc]) s -= A->val[p] * x[cc];
            else { const int64_t d = llabs(perm[cc] - u); if (d > bw) bw = d; }
        }
        rhs[u] = s;
    }
    const int64_t ld = bw + 1;
    double *L = (double *)calloc((size_t)(nf > 0 ? nf : 1) * (size_t)ld, sizeof(double));
    /* lower band: L[(i - j) + ld * j] = A(i, j) for 0 <= i - j <= bw */
    for (int64_t u = 0; u < nf; u++) {
        const int64_t r = node_of[u];
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; p++) {
            const int64_t cc = A->col[p];
            if (dmask[cc]) continue;
            const int64_t v = perm[cc];
            if (u >= v) L[(u - v) + ld * v] = A->val[p];
        }
    }
    int status = 0;
    for (int64_t j = 0; j < nf && status == 0; j++) {
        const int64_t k0 = (j - bw > 0) ? j - bw : 0;
        double s = L[ld * j];
        for (int64_t k = k0; k < j; k++) { const double l = L[(j - k) + ld * k]; s -= l * l; }
        if (!(s > 0.0)) { status = -4; break; }
        const double d = sqrt(s);
        L[ld * j] = d;
        const int64_t iend = (j + bw < nf - 1) ? j + bw : nf - 1;
        #pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i <= iend; i++) {
            const int64_t kk0 = (i - bw > 0) ? i - bw : 0;
            double t = L[(i - j) + ld * j];
            for (int64_t k = kk0; k < j; k++) t -= L[(i - k) + ld * k] * L[(j - k) + ld * k];
            L[(i - j) + ld * j] = t / d;
        }
    }
    if (status == 0) {
        for (int64_t i = 0; i < nf; i++) {        /* L y = rhs */
            const int64_t k0 = (i - bw > 0) ? i - bw : 0;
            double s = rhs[i];
            for (int64_t k = k0; k < i; k++) s -= L[(i - k) + ld * k] * rhs[k];
            rhs[i] = s / L[ld * i];
        }
        for (int64_t i = nf - 1; i >= 0; i--) {   /* L^T x = y */
            const int64_t kend = (i + bw < nf - 1) ? i + bw : nf - 1;
            double s = rhs[i];
            for (int64_t k = i + 1; k <= kend; k++) s -= L[(k - i) + ld * i] * rhs[k];
            rhs[i] = s / L[ld * i];
        }
        for (int64_t u = 0; u < nf; u++) x[node_of[u]] = rhs[u];
    }
    free(perm); free(node_of); free(rhs); free(L);
    return status;
}

/* ------------------------------------------------------------------------ */
/* EXP_finite (Section 4.3): third-order initial guess W on level l from      */
/* U1 = u_{l-1} and U0 = u_{l-2}.  Fine dims nx,ny,nz are level l's.          */
/* ------------------------------------------------------------------------ */

/* Serendipity shape function of node (am,bm,cm) in {0,2,4}^3 (one of the 20)
 * at natural coordinates (xi,eta,zeta) in [-1,1]^3 (eq. inter). */
static double serendipity_N(int am, int bm, int cm, double xi, double eta, double zeta) {
    const double xm = am / 2 - 1, ym = bm / 2 - 1, zm = cm / 2 - 1;
    if (am != 2 && bm != 2 && cm != 2)
        return 0.125 * (1.0 + xm * xi) * (1.0 + ym * eta) * (1.0 + zm * zeta) *
               (xm * xi + ym * eta + zm * zeta - 2.0);
    if (am == 2) return 0.25 * (1.0 - xi * xi) * (1.0 + ym * eta) * (1.0 + zm * zeta);
    if (bm == 2) return 0.25 * (1.0 - eta * eta) * (1.0 + xm * xi) * (1.0 + zm * zeta);
    return 0.25 * (1.0 - zeta * zeta) * (1.0 + xm * xi) * (1.0 + ym * eta);
}

double orc_serendipity_weight(int am, int bm, int cm, double xi, double eta, double zeta) {
    return serendipity_N(am, bm, cm, xi, eta, zeta);
}

/* W at fine node (i,j,k) of level l (not overwritten by g_D here). */
double orc_exp_finite_node(int64_t nx, int64_t ny, int64_t nz, const double *U1, const double *U0,
                           int64_t i, int64_t j, int64_t k) {
    const int64_t NX = nx / 4, NY = ny / 4, NZ = nz / 4;              /* level l-2 elements */
    const int64_t I = (i / 4 < NX - 1) ? i / 4 : NX - 1;              /* owner coarse element */
    const int64_t J = (j / 4 < NY - 1) ? j / 4 : NY - 1;
    const int64_t K = (k / 4 < NZ - 1) ? k / 4 : NZ - 1;
    const int a = (int)(i - 4 * I), b = (int)(j - 4 * J), c = (int)(k - 4 * K);
    const int64_t n1x = nx / 2 + 1, n1y = ny / 2 + 1;                 /* level l-1 node dims */
    const int64_t n0x = nx / 4 + 1, n0y = ny / 4 + 1;                 /* level l-2 node dims */
#define ORC_U1(aa, bb, cc) U1[(2 * I + (aa) / 2) + n1x * ((2 * J + (bb) / 2) + n1y * (2 * K + (cc) / 2))]
#define ORC_U0(aa, bb, cc) U0[(I + (aa) / 4) + n0x * ((J + (bb) / 4) + n0y * (K + (cc) / 4))]
    /* W_m at the 20 nodes, indexed by local offsets */
    double Wm[5][5][5];
    for (int cc = 0; cc <= 4; cc += 2)
        for (int bb = 0; bb <= 4; bb += 2)
            for (int aa = 0; aa <= 4; aa += 2) {
                const int twos = (aa == 2) + (bb == 2) + (cc == 2);
                if (twos == 0) {                                    /* corner: eq. jiedian */
                    Wm[aa][bb][cc] = (5.0 * ORC_U1(aa, bb, cc) - ORC_U0(aa, bb, cc)) / 4.0;
                } else if (twos == 1) {                             /* mid-edge: eq. zhongdian */
                    int a0 = aa, a1 = aa, b0 = bb, b1 = bb, c0 = cc, c1 = cc;
                    if (aa == 2) { a0 = 0; a1 = 4; }
                    if (bb == 2) { b0 = 0; b1 = 4; }
                    if (cc == 2) { c0 = 0; c1 = 4; }
                    Wm[aa][bb][cc] = ORC_U1(aa, bb, cc) +
                        (ORC_U1(a0, b0, c0) - ORC_U0(a0, b0, c0) + ORC_U1(a1, b1, c1) - ORC_U0(a1, b1, c1)) / 8.0;
                }
            }
#undef ORC_U1
#undef ORC_U0
    const int twos = (a == 2) + (b == 2) + (c == 2);
    const int on20 = (a % 2 == 0) && (b % 2 == 0) && (c % 2 == 0) && twos <= 1;
    if (on20) return Wm[a][b][c];
    /* the other 105 nodes: tri-quadratic serendipity interpolation (eq. inter),
     * summed over the 20 nodes in the paper's node-number order 1 + a + 5b + 25c */
    const double xi = a / 2.0 - 1.0, eta = b / 2.0 - 1.0, zeta = c / 2.0 - 1.0;
    double s = 0.0;
    for (int cc = 0; cc <= 4; cc += 2)
        for (int bb = 0; bb <= 4; bb += 2)
            for (int aa = 0; aa <= 4; aa += 2) {
                if ((aa == 2) + (bb == 2) + (cc == 2) > 1) continue;
                s += serendipity_N(aa, bb, cc, xi, eta, zeta) * Wm[aa][bb][cc];
            }
    return s;
}

/* Variant of the Remark after eq. inter: the 6 face centres are the mean of
 * eq. zhongdian along the face's 2 diagonals, the body centre the mean along the
 * 4 space diagonals, and the other 98 fine nodes come from tri-quadratic
 * Lagrange interpolation of the 27 values.  Arguments as orc_exp_finite_node. */
static double lagrange_q(int m, double t) {           /* 1-D quadratic Lagrange basis at -1, 0, 1 */
    if (m == 0) return 0.5 * t * (t - 1.0);
    if (m == 1) return 1.0 - t * t;
    return 0.5 * t * (t + 1.0);
}

double orc_exp_finite_node_lagrange27(int64_t nx, int64_t ny, int64_t nz, const double *U1, const double *U0,
                                      int64_t i, int64_t j, int64_t k) {
    const int64_t NX = nx / 4, NY = ny / 4, NZ = nz / 4;
    const int64_t I = (i / 4 < NX - 1) ? i / 4 : NX - 1;
    const int64_t J = (j / 4 < NY - 1) ? j / 4 : NY - 1;
    const int64_t K = (k / 4 < NZ - 1) ? k / 4 : NZ - 1;
    const int a = (int)(i - 4 * I), b = (int)(j - 4 * J), c = (int)(k - 4 * K);
    const int64_t n1x = nx / 2 + 1, n1y = ny / 2 + 1;
    const int64_t n0x = nx / 4 + 1, n0y = ny / 4 + 1;
#define L_U1(aa, bb, cc) U1[(2 * I + (aa) / 2) + n1x * ((2 * J + (bb) / 2) + n1y * (2 * K + (cc) / 2))]
#define L_U0(aa, bb, cc) U0[(I + (aa) / 4) + n0x * ((J + (bb) / 4) + n0y * (K + (cc) / 4))]
#define L_DEL(aa, bb, cc) (L_U1(aa, bb, cc) - L_U0(aa, bb, cc))
    double V[3][3][3];
    for (int cc = 0; cc <= 4; cc += 2)
        for (int bb = 0; bb <= 4; bb += 2)
            for (int aa = 0; aa <= 4; aa += 2) {
                const int o[3] = {aa, bb, cc};
                int mid[3], nmid = 0;
                for (int ax = 0; ax < 3; ax++) if (o[ax] == 2) mid[nmid++] = ax;
                if (nmid == 0) {                                   /* corner: eq. jiedian */
                    V[aa / 2][bb / 2][cc / 2] = (5.0 * L_U1(aa, bb, cc) - L_U0(aa, bb, cc)) / 4.0;
                    continue;
                }
                /* eq. zhongdian along each of the 1, 2 or 4 diagonals through this
                 * node (step +2 on the first mid axis, +-2 on the others), averaged */
                const int ndiag = 1 << (nmid - 1);
                double sum = 0.0;
                for (int s = 0; s < ndiag; s++) {
                    int d[3] = {0, 0, 0};
                    d[mid[0]] = 2;
                    for (int t = 1; t < nmid; t++) d[mid[t]] = ((s >> (t - 1)) & 1) ? -2 : 2;
                    sum += L_U1(aa, bb, cc) +
                           (L_DEL(aa - d[0], bb - d[1], cc - d[2]) + L_DEL(aa + d[0], bb + d[1], cc + d[2])) / 8.0;
                }
                V[aa / 2][bb / 2][cc / 2] = sum / (double)ndiag;
            }
#undef L_U1
#undef L_U0
#undef L_DEL
    if (a % 2 == 0 && b % 2 == 0 && c % 2 == 0) return V[a / 2][b / 2][c / 2];
    const double xi = a / 2.0 - 1.0, eta = b / 2.0 - 1.0, zeta = c / 2.0 - 1.0;
    double s = 0.0;
    for (int cc = 0; cc < 3; cc++)
        for (int bb = 0; bb < 3; bb++)
            for (int aa = 0; aa < 3; aa++)
                s += lagrange_q(aa, xi) * lagrange_q(bb, eta) * lagrange_q(cc, zeta) * V[aa][bb][cc];
    return s;
}

/* W on every node of level l (the extrapolation/interpolation output itself;
 * the cascade imposes g_D on Dirichlet nodes before JCG starts).
 * variant 0 = 20-node serendipity (Section 4.3), 1 = the 27-node Lagrange
 * variant of the Remark. */
void orc_exp_finite(const orc_grid *g, const double *U1, const double *U0, double *W, int variant) {
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k <= g->nz; k++)
        for (int64_t j = 0; j <= g->ny; j++)
            for (int64_t i = 0; i <= g->nx; i++)
                W[nid(g, i, j, k)] = variant ? orc_exp_finite_node_lagrange27(g->nx, g->ny, g->nz, U1, U0, i, j, k)
                                             : orc_exp_finite_node(g->nx, g->ny, g->nz, U1, U0, i, j, k);
}

void orc_exp_finite_points(int64_t nx, int64_t ny, int64_t nz, const double *U1, const double *U0,
                           const int64_t *pts, int64_t npts, double *out, int variant) {
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; t++) {
        const int64_t r = pts[t];
        const int64_t i = r % (nx + 1), j = (r / (nx + 1)) % (ny + 1), k = r / ((nx + 1) * (ny + 1));
        out[t] = variant ? orc_exp_finite_node_lagrange27(nx, ny, nz, U1, U0, i, j, k)
                         : orc_exp_finite_node(nx, ny, nz, U1, U0, i, j, k);
    }
}

/* ------------------------------------------------------------------------ */
/* EXP_true (Section 4.2.1 and the end of Section 4.3): fourth-order         */
/* extrapolation on level l from U1 = u_l and U0 = u_{l-1}.                  */
/* Coarse nodes: eq. t1.  Edge midpoints: eq. chenlin.  Face centres: mean of */
/* chenlin along the 2 face diagonals; body centres: mean over the 4 space   */
/* diagonals.                                                                 */
/* ------------------------------------------------------------------------ */
double orc_exp_true_node(int64_t nx, int64_t ny, int64_t nz, const double *U1, const double *U0,
                         int64_t i, int64_t j, int64_t k) {
    const int64_t m1x = nx + 1, m1y = ny + 1;
    const int64_t m0x = nx / 2 + 1, m0y = ny / 2 + 1;
    (void)nz;
#define T_D(a, b, c) (U1[(a) + m1x * ((b) + m1y * (c))] - U0[(a) / 2 + m0x * ((b) / 2 + m0y * ((c) / 2))])
    const int64_t p[3] = {i, j, k};
    int oddax[3], nodd = 0;
    for (int ax = 0; ax < 3; ax++) if (p[ax] & 1) oddax[nodd++] = ax;
    const double u1 = U1[i + m1x * (j + m1y * k)];
    if (nodd == 0)                                          /* coarse node: eq. t1 */
        return (4.0 * u1 - U0[i / 2 + m0x * (j / 2 + m0y * (k / 2))]) / 3.0;
    /* The node is the midpoint of 1 edge (one odd axis), 2 face diagonals (two
     * odd axes) or 4 space diagonals (three odd axes).  A diagonal has step +1
     * on the first odd axis and +-1 on the others; its endpoints are the coarse
     * nodes p - step and p + step.  Apply eq. chenlin along each and average. */
    const int ndiag = 1 << (nodd - 1);
    double sum = 0.0;
    for (int s = 0; s < ndiag; s++) {
        int64_t d[3] = {0, 0, 0};
        d[oddax[0]] = 1;
        for (int t = 1; t < nodd; t++) d[oddax[t]] = ((s >> (t - 1)) & 1) ? -1 : 1;
        const double da = T_D(i - d[0], j - d[1], k - d[2]);
        const double db = T_D(i + d[0], j + d[1], k + d[2]);
        sum += u1 + (da + db) / 6.0;
    }
#undef T_D
    return sum / (double)ndiag;
}

void orc_exp_true(const orc_grid *g, const double *U1, const double *U0, double *Ut) {
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k <= g->nz; k++)
        for (int64_t j = 0; j <= g->ny; j++)
            for (int64_t i = 0; i <= g->nx; i++)
                Ut[nid(g, i, j, k)] = orc_exp_true_node(g->nx, g->ny, g->nz, U1, U0, i, j, k);
}

void orc_exp_true_points(int64_t nx, int64_t ny, int64_t nz, const double *U1, const double *U0,
                         const int64_t *pts, int64_t npts, double *out) {
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; t++) {
        const int64_t r = pts[t];
        const int64_t i = r % (nx + 1), j = (r / (nx + 1)) % (ny + 1), k = r / ((nx + 1) * (ny + 1));
        out[t] = orc_exp_true_node(nx, ny, nz, U1, U0, i, j, k);
    }
}

/* ------------------------------------------------------------------------ */
/* Row-by-row operator for sampled checks at sizes where CSR does not fit:   */
/* out[t] = (A v)_r for r = pts[t] (0 on Dirichlet rows), element matrices    */
/* integrated on the fly exactly as in orc_assemble.                         */
/* ------------------------------------------------------------------------ */
void orc_apply_rows(const orc_grid *g, const double *beta, const double *const *alpha,
                    const double *v, const int64_t *pts, int64_t npts, double *out) {
    double K[64];
    orc_element_stiffness(g->hx, g->hy, g->hz, K);
    const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; t++) {
        double M[16];
        const int64_t r = pts[t];
        const int64_t i = r % (nx + 1), j = (r / (nx + 1)) % (ny + 1), k = r / ((nx + 1) * (ny + 1));
        if (is_dirichlet(g, i, j, k)) { out[t] = 0.0; continue; }
        double s = 0.0;
        for (int64_t ke = k - 1; ke <= k; ke++) {
            if (ke < 0 || ke >= nz) continue;
            for (int64_t je = j - 1; je <= j; je++) {
                if (je < 0 || je >= ny) continue;
                for (int64_t ie = i - 1; ie <= i; ie++) {
                    if (ie < 0 || ie >= nx) continue;
                    const double b = beta[ie + nx * (je + ny * ke)];
                    const int a = (int)((i - ie) + 2 * (j - je) + 4 * (k - ke));
                    for (int c = 0; c < 8; c++)
                        s += b * K[a * 8 + c] * v[nid(g, ie + (c & 1), je + ((c >> 1) & 1), ke + ((c >> 2) & 1))];
                }
            }
        }
        for (int f = 0; f < 6; f++) {
            if (g->face_type[f] != 1 || alpha == NULL || alpha[f] == NULL) continue;
            int pax, qax, nax; int64_t nfix, np, nq; double hp, hq;
            face_axes(g, f, &pax, &qax, &nax, &nfix, &np, &nq, &hp, &hq);
            const int64_t idx[3] = {i, j, k};
            if (idx[nax] != nfix) continue;
            orc_face_mass(hp, hq, M);
            const int64_t pi = idx[pax], qi = idx[qax];
            for (int64_t eq = qi - 1; eq <= qi; eq++) {
                if (eq < 0 || eq >= nq) continue;
                for (int64_t ep = pi - 1; ep <= pi; ep++) {
                    if (ep < 0 || ep >= np) continue;
                    const double al = alpha[f][ep + np * eq];
                    const int a = (int)((pi - ep) + 2 * (qi - eq));
                    for (int c = 0; c < 4; c++) {
                        int64_t cidx[3] = {i, j, k};
                        cidx[pax] = ep + (c & 1);
                        cidx[qax] = eq + ((c >> 1) & 1);
                        s += al * M[a * 4 + c] * v[nid(g, cidx[0], cidx[1], cidx[2])];
                    }
                }
            }
        }
        out[t] = s;
    }
}
