/*
 * bb_oracle.c -- plain, slow, obviously-correct FP64 CPU solvers for batches
 * of banded systems that all share one left-hand-side matrix.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no source, header, table or helper with the GPU library; the two
 * meet only through the seeded input generators.
 *
 * Source of every formula: Carroll, Gloster, Bustamante, O Naraigh,
 * "A Batched GPU Methodology for Numerical Solutions of Partial Differential
 * Equations" (arXiv:2107.05395).  Each function names the passage it follows.
 *
 * Conventions
 *  - IEEE double throughout, true divisions as the paper writes them (no
 *    stored reciprocals), no -ffast-math.
 *  - The paper numbers rows 1..N; here rows are 0..n-1, so the paper's q_i is
 *    q[i-1] below.
 *  - Tridiagonal row i:  a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i].
 *    Non-cyclic: a[0] and c[n-1] are ignored.  Cyclic (indices mod n):
 *    a[0] is the top-right corner A[0][n-1], c[n-1] the bottom-left A[n-1][0].
 *  - Pentadiagonal row i:
 *        a[i] x[i-2] + b[i] x[i-1] + c[i] x[i] + d[i] x[i+1] + e[i] x[i+2] = f[i].
 *    Non-cyclic: a[0], a[1], b[0], d[n-1], e[n-2], e[n-1] are ignored.
 *    Cyclic (indices mod n): those six entries are the wrap-around corners.
 *  - Batched ("interleaved") storage: element i of system k sits at
 *    [i*ld + k], 0 <= k < m <= ld  (Section 2, interleaved layout figure).
 *  - Return value: 0 on success, 1 when a pivot is zero or not finite (the
 *    method does not pivot), 2 when a Sherman-Morrison / Woodbury capacitance
 *    is singular, 3 for bad sizes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define ERR_PIVOT 1
#define ERR_CAPACITANCE 2
#define ERR_SIZE 3

static int bad_pivot(double p) { return p == 0.0 || !isfinite(p); }

/* ------------------------------------------------------------------------ */
/* Tridiagonal: the Thomas algorithm, Section 3.1 (pre-factorisation, forward
 * sweep, backward sweep).  The printed backward equation drops x_{i+1}; the
 * appendix's batched listing has the intended x_i = d^_i - c^_i x_{i+1}, which
 * is what is used here.  Workspace: 2n doubles.                              */
int oracle_tri_solve(int64_t n, const double *a, const double *b, const double *c,
                     const double *d, double *x, double *work)
{
    if (n < 1) return ERR_SIZE;
    double *chat = work, *bhat = work + n;
    /* pre-factorisation: c^_1 = c_1/b_1; b^_i = b_i - a_i c^_{i-1}; c^_i = c_i/b^_i */
    bhat[0] = b[0];
    if (bad_pivot(bhat[0])) return ERR_PIVOT;
    chat[0] = (n > 1) ? c[0] / bhat[0] : 0.0;
    for (int64_t i = 1; i < n; ++i) {
        bhat[i] = b[i] - a[i] * chat[i - 1];
        if (bad_pivot(bhat[i])) return ERR_PIVOT;
        chat[i] = (i < n - 1) ? c[i] / bhat[i] : 0.0;
    }
    /* forward sweep: d^_1 = d_1/b_1; d^_i = (d_i - a_i d^_{i-1}) / b^_i */
    x[0] = d[0] / bhat[0];
    for (int64_t i = 1; i < n; ++i)
        x[i] = (d[i] - a[i] * x[i - 1]) / bhat[i];
    /* backward sweep: x_N = d^_N; x_i = d^_i - c^_i x_{i+1} */
    for (int64_t i = n - 2; i >= 0; --i)
        x[i] = x[i] - chat[i] * x[i + 1];
    return OK;
}

/* ------------------------------------------------------------------------ */
/* Pentadiagonal: the LR factorisation A = L R, then L g = f, then R x = g,
 * Section 4.1.  The paper lists the factorisation as steps 1-14 with rows 1,
 * 2, N-1 and N written out; that list is exactly the single loop below once
 * every entry that falls outside the matrix is taken as zero (a_1 = a_2 =
 * b_1 = 0, d_N = e_{N-1} = e_N = 0, and gamma, delta of rows before the first
 * are zero).  eps_i = a_i (step 14).  Workspace: 4n doubles.                */
int oracle_penta_solve(int64_t n, const double *a, const double *b, const double *c,
                       const double *d, const double *e, const double *f, double *x,
                       double *work)
{
    if (n < 1) return ERR_SIZE;
    double *alpha = work, *beta = work + n, *gamma = work + 2 * n, *delta = work + 3 * n;
    for (int64_t i = 0; i < n; ++i) {
        const double ai = (i >= 2) ? a[i] : 0.0;          /* eps_i */
        const double bi = (i >= 1) ? b[i] : 0.0;
        const double di = (i <= n - 2) ? d[i] : 0.0;
        const double ei = (i <= n - 3) ? e[i] : 0.0;
        const double gm2 = (i >= 2) ? gamma[i - 2] : 0.0;
        const double gm1 = (i >= 1) ? gamma[i - 1] : 0.0;
        const double dm2 = (i >= 2) ? delta[i - 2] : 0.0;
        const double dm1 = (i >= 1) ? delta[i - 1] : 0.0;
        beta[i] = bi - ai * gm2;                          /* beta_i  = b_i - a_i gamma_{i-2} */
        alpha[i] = c[i] - ai * dm2 - beta[i] * gm1;       /* alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1} */
        if (bad_pivot(alpha[i])) return ERR_PIVOT;
        gamma[i] = (di - beta[i] * dm1) / alpha[i];       /* gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i */
        delta[i] = ei / alpha[i];                         /* delta_i = e_i / alpha_i */
    }
    /* L g = f: g_i = (f_i - eps_i g_{i-2} - beta_i g_{i-1}) / alpha_i */
    for (int64_t i = 0; i < n; ++i) {
        const double ai = (i >= 2) ? a[i] : 0.0;
        const double g2 = (i >= 2) ? x[i - 2] : 0.0;
        const double g1 = (i >= 1) ? x[i - 1] : 0.0;
        x[i] = (f[i] - ai * g2 - beta[i] * g1) / alpha[i];
    }
    /* R x = g: x_N = g_N; x_{N-1} = g_{N-1} - gamma_{N-1} x_N;
       x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2} */
    for (int64_t i = n - 2; i >= 0; --i) {
        const double x2 = (i + 2 < n) ? x[i + 2] : 0.0;
        x[i] = x[i] - gamma[i] * x[i + 1] - delta[i] * x2;
    }
    return OK;
}

/* ------------------------------------------------------------------------ */
/* Periodic tridiagonal by Sherman-Morrison, Section 3.3, generalised from the
 * constant bands there to row-dependent ones: A = A' + U V^T with
 *   U = (-b_1, 0, ..., 0, c_N^wrap)^T,  V = (1, 0, ..., 0, -a_1^wrap / b_1)^T,
 *   A'_11 = 2 b_1,  A'_NN = b_N + a_1^wrap c_N^wrap / b_1,
 * solve A' y = d and A' z = U, then x = y - (V.y)/(1 + V.z) z.
 * n >= 3.  Workspace: 6n doubles.                                            */
int oracle_tri_cyclic_solve(int64_t n, const double *a, const double *b, const double *c,
                            const double *d, double *x, double *work)
{
    if (n < 3) return ERR_SIZE;
    if (bad_pivot(b[0])) return ERR_PIVOT;
    double *bp = work, *u = work + n, *z = work + 2 * n, *tw = work + 3 * n; /* tw: 2n */
    double *y = work + 5 * n;                                                  /* n */
    const double a_wrap = a[0], c_wrap = c[n - 1];
    const double v_last = -a_wrap / b[0];
    for (int64_t i = 0; i < n; ++i) { bp[i] = b[i]; u[i] = 0.0; }
    bp[0] = 2.0 * b[0];
    bp[n - 1] = b[n - 1] + a_wrap * c_wrap / b[0];
    u[0] = -b[0];
    u[n - 1] = c_wrap;
    int s = oracle_tri_solve(n, a, bp, c, d, y, tw);
    if (s) return s;
    s = oracle_tri_solve(n, a, bp, c, u, z, tw);
    if (s) return s;
    const double vy = y[0] + v_last * y[n - 1];
    const double vz = z[0] + v_last * z[n - 1];
    const double den = 1.0 + vz;
    if (bad_pivot(den)) return ERR_CAPACITANCE;
    const double fac = vy / den;
    for (int64_t i = 0; i < n; ++i) x[i] = y[i] - fac * z[i];
    return OK;
}

/* ------------------------------------------------------------------------ */
/* Periodic pentadiagonal.  Section 5.1 builds this matrix (the Cahn-Hilliard
 * LHS) and only cites outside work for its solution.  Reading used here: the
 * rank-2 Woodbury analogue of the periodic tridiagonal treatment above.  With
 *   T = A[0:2,0:2] (top-left block), B = A[0:2,n-2:n] (top-right corners),
 *   C = A[n-2:n,0:2] (bottom-left corners),
 *   U = [-T; 0; C] (n x 2),  V^T = [I_2, 0, -T^{-1} B] (2 x n),
 * A' = A - U V^T is pentadiagonal without corners (top-left block 2T,
 * bottom-right block A_BR + C T^{-1} B).  Then y = A'^{-1} f, Z = A'^{-1} U,
 * H = (I_2 + V^T Z)^{-1}, x = y - Z H V^T y.  With 1x1 blocks this is the
 * tridiagonal formula above.  n >= 5.  Workspace: 14n doubles.             */
static int inv2(const double m[4], double out[4])
{
    const double det = m[0] * m[3] - m[1] * m[2];
    if (bad_pivot(det)) return 1;
    out[0] = m[3] / det;  out[1] = -m[1] / det;
    out[2] = -m[2] / det; out[3] = m[0] / det;
    return 0;
}

int oracle_penta_cyclic_solve(int64_t n, const double *a, const double *b, const double *c,
                              const double *d, const double *e, const double *f, double *x,
                              double *work)
{
    if (n < 5) return ERR_SIZE;
    /* the dense 2x2 corner blocks, rows/cols as in the comment above */
    const double T[4] = { c[0], d[0], b[1], c[1] };
    const double B[4] = { a[0], b[0], 0.0, a[1] };              /* A[0][n-2], A[0][n-1]; A[1][n-2], A[1][n-1] */
    const double C[4] = { e[n - 2], 0.0, d[n - 1], e[n - 1] };  /* A[n-2][0], A[n-2][1]; A[n-1][0], A[n-1][1] */
    double Ti[4], W[4];
    if (inv2(T, Ti)) return ERR_PIVOT;
    /* W = T^{-1} B */
    W[0] = Ti[0] * B[0] + Ti[1] * B[2]; W[1] = Ti[0] * B[1] + Ti[1] * B[3];
    W[2] = Ti[2] * B[0] + Ti[3] * B[2]; W[3] = Ti[2] * B[1] + Ti[3] * B[3];
    /* CW = C T^{-1} B, added to the bottom-right block of A' */
    const double CW[4] = { C[0] * W[0] + C[1] * W[2], C[0] * W[1] + C[1] * W[3],
                           C[2] * W[0] + C[3] * W[2], C[2] * W[1] + C[3] * W[3] };

    double *pa = work, *pb = work + n, *pc = work + 2 * n, *pd = work + 3 * n, *pe = work + 4 * n;
    double *u0 = work + 5 * n, *u1 = work + 6 * n, *z0 = work + 7 * n, *z1 = work + 8 * n;
    double *y = work + 9 * n;
    double *tw = work + 10 * n; /* 4n needed; caller gives 14n in total */
    for (int64_t i = 0; i < n; ++i) {
        pa[i] = a[i]; pb[i] = b[i]; pc[i] = c[i]; pd[i] = d[i]; pe[i] = e[i];
        u0[i] = 0.0; u1[i] = 0.0;
    }
    /* A' top-left block 2T: entries (0,0),(0,1),(1,0),(1,1) */
    pc[0] = 2.0 * T[0]; pd[0] = 2.0 * T[1]; pb[1] = 2.0 * T[2]; pc[1] = 2.0 * T[3];
    /* A' bottom-right block A_BR + C T^{-1} B: (n-2,n-2),(n-2,n-1),(n-1,n-2),(n-1,n-1) */
    pc[n - 2] = c[n - 2] + CW[0]; pd[n - 2] = d[n - 2] + CW[1];
    pb[n - 1] = b[n - 1] + CW[2]; pc[n - 1] = c[n - 1] + CW[3];
    /* U columns: [-T; 0; C] */
    u0[0] = -T[0]; u1[0] = -T[1];
    u0[1] = -T[2]; u1[1] = -T[3];
    u0[n - 2] = C[0]; u1[n - 2] = C[1];
    u0[n - 1] = C[2]; u1[n - 1] = C[3];

    int s;
    if ((s = oracle_penta_solve(n, pa, pb, pc, pd, pe, f, y, tw))) return s;
    if ((s = oracle_penta_solve(n, pa, pb, pc, pd, pe, u0, z0, tw))) return s;
    if ((s = oracle_penta_solve(n, pa, pb, pc, pd, pe, u1, z1, tw))) return s;

    /* V^T v = v[0:2] - W v[n-2:n] */
    const double vy0 = y[0] - (W[0] * y[n - 2] + W[1] * y[n - 1]);
    const double vy1 = y[1] - (W[2] * y[n - 2] + W[3] * y[n - 1]);
    const double I_VZ[4] = {
        1.0 + z0[0] - (W[0] * z0[n - 2] + W[1] * z0[n - 1]), z1[0] - (W[0] * z1[n - 2] + W[1] * z1[n - 1]),
        z0[1] - (W[2] * z0[n - 2] + W[3] * z0[n - 1]), 1.0 + z1[1] - (W[2] * z1[n - 2] + W[3] * z1[n - 1]) };
    double H[4];
    if (inv2(I_VZ, H)) return ERR_CAPACITANCE;
    const double s0 = H[0] * vy0 + H[1] * vy1;
    const double s1 = H[2] * vy0 + H[3] * vy1;
    for (int64_t i = 0; i < n; ++i) x[i] = y[i] - (z0[i] * s0 + z1[i] * s1);
    return OK;
}

/* ------------------------------------------------------------------------ */
/* Transposed bands.  A^T of a tridiagonal matrix has sub-diagonal c_{i-1},
 * diagonal b_i and super-diagonal a_{i+1}; of a pentadiagonal one, bands
 * (e_{i-2}, d_{i-1}, c_i, b_{i+1}, a_{i+2}).  Indices are taken mod n, which
 * also carries the corner entries of a cyclic matrix over correctly.  The
 * adjoint solve A^T lam = g is then an ordinary solve with these bands.     */
static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

void oracle_tri_transpose_bands(int64_t n, const double *a, const double *b, const double *c,
                                double *at, double *bt, double *ct)
{
    for (int64_t i = 0; i < n; ++i) {
        at[i] = c[wrap(i - 1, n)];
        bt[i] = b[i];
        ct[i] = a[wrap(i + 1, n)];
    }
}

void oracle_penta_transpose_bands(int64_t n, const double *a, const double *b, const double *c,
                                  const double *d, const double *e, double *at, double *bt,
                                  double *ct, double *dt, double *et)
{
    for (int64_t i = 0; i < n; ++i) {
        at[i] = e[wrap(i - 2, n)];
        bt[i] = d[wrap(i - 1, n)];
        ct[i] = c[i];
        dt[i] = b[wrap(i + 1, n)];
        et[i] = a[wrap(i + 2, n)];
    }
}

/* ------------------------------------------------------------------------ */
/* Batched drivers: one system at a time, column k gathered from the
 * interleaved array, solved, scattered back.  OpenMP splits the systems over
 * the host's cores; each system is still solved by one plain sequential call.
 * kind: 0 tri, 1 tri cyclic, 2 penta, 3 penta cyclic.
 * Returns the first nonzero per-system status, or 0.                       */
int oracle_solve_batch(int kind, int64_t n, int64_t m, int64_t ld, const double *a,
                       const double *b, const double *c, const double *d, const double *e,
                       const double *rhs, double *x)
{
    if (n < 1 || m < 0 || ld < m) return ERR_SIZE;
    int status = OK;
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (size_t)n * 16);
        double *sol = col + n, *work = col + 2 * n;   /* 14n of workspace */
        int my = OK;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            for (int64_t i = 0; i < n; ++i) col[i] = rhs[i * ld + k];
            int s;
            switch (kind) {
            case 0: s = oracle_tri_solve(n, a, b, c, col, sol, work); break;
            case 1: s = oracle_tri_cyclic_solve(n, a, b, c, col, sol, work); break;
            case 2: s = oracle_penta_solve(n, a, b, c, d, e, col, sol, work); break;
            case 3: s = oracle_penta_cyclic_solve(n, a, b, c, d, e, col, sol, work); break;
            default: s = ERR_SIZE;
            }
            if (s && !my) my = s;
            for (int64_t i = 0; i < n; ++i) x[i * ld + k] = s ? NAN : sol[i];
        }
        free(col);
#pragma omp critical
        { if (my && !status) status = my; }
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Band gradients.  For A x = b with loss L and adjoint lam = A^{-T} dL/dx, the
 * gradient with respect to a matrix entry is dL/dA_ij = -lam_i x_j; summed
 * over the batch for each entry of each band:
 *   grad[band][i] = - sum_k lam[i,k] * x[i + off(band), k],
 * off = -1, 0, +1 (tri; bands a, b, c) or -2..+2 (penta; a..e).  Entries that
 * fall outside the matrix get 0, unless cyclic, where the index wraps mod n.
 * nb = 3 or 5; grad is nb*n doubles, written (not accumulated).           */
void oracle_band_grad(int nb, int cyclic, int64_t n, int64_t m, int64_t ld,
                      const double *lam, const double *x, double *grad)
{
    const int half = nb / 2;
    for (int band = 0; band < nb; ++band) {
        const int off = band - half;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t j = i + off;
            double s = 0.0;
            if (j < 0 || j >= n) {
                if (!cyclic) { grad[band * n + i] = 0.0; continue; }
                j = wrap(j, n);
            }
            for (int64_t k = 0; k < m; ++k) s += lam[i * ld + k] * x[j * ld + k];
            grad[band * n + i] = -s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One semi-implicit Cahn-Hilliard step, Section 5.1:
 *   C^{n+1} + dt*gamma*d4 C^{n+1} = C^n + dt*d2 (C^3 - C)^n,  periodic,
 * with second-order central differences.  Matrix bands a = e = sigma,
 * b = d = -4 sigma, c = 1 + 6 sigma, sigma = gamma dt / dx^4.  Right-hand
 * side f_i = C_i + alpha (N_{i-1} - 2 N_i + N_{i+1}), N = C^3 - C,
 * alpha = dt / dx^2.  (The printed f_i leaves out C_i^n, which the scheme
 * itself requires; the printed fourth-difference stencil's centre weight
 * reads 1 where the matrix entry 1 + 6 sigma implies 6.)  Uses the periodic
 * pentadiagonal solver above.                                              */
int oracle_ch_step_batch(int64_t n, int64_t m, int64_t ld, double sigma, double alpha,
                         const double *c_in, double *c_out)
{
    if (n < 5 || m < 0 || ld < m) return ERR_SIZE;
    double *band = (double *)malloc(sizeof(double) * (size_t)n * 5);
    double *ba = band, *bb = band + n, *bc = band + 2 * n, *bd = band + 3 * n, *be = band + 4 * n;
    for (int64_t i = 0; i < n; ++i) {
        ba[i] = sigma; bb[i] = -4.0 * sigma; bc[i] = 1.0 + 6.0 * sigma;
        bd[i] = -4.0 * sigma; be[i] = sigma;
    }
    int status = OK;
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (size_t)n * 18);
        double *nl = col + n, *f = col + 2 * n, *sol = col + 3 * n, *work = col + 4 * n;
        int my = OK;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            for (int64_t i = 0; i < n; ++i) {
                col[i] = c_in[i * ld + k];
                nl[i] = col[i] * col[i] * col[i] - col[i];
            }
            for (int64_t i = 0; i < n; ++i)
                f[i] = col[i] + alpha * (nl[wrap(i - 1, n)] - 2.0 * nl[i] + nl[wrap(i + 1, n)]);
            int s = oracle_penta_cyclic_solve(n, ba, bb, bc, bd, be, f, sol, work);
            if (s && !my) my = s;
            for (int64_t i = 0; i < n; ++i) c_out[i * ld + k] = s ? NAN : sol[i];
        }
        free(col);
#pragma omp critical
        { if (my && !status) status = my; }
    }
    free(band);
    return status;
}

/* ------------------------------------------------------------------------ */
/* One-sided fifth-order WENO derivative for Hamilton-Jacobi equations (Jiang
 * and Peng; the scheme the paper cites for the advection term of the forced
 * Cahn-Hilliard equation), undivided (it returns dx times the derivative) on
 * a periodic grid function phi.  plus != 0: the right-biased derivative,
 * from phi_{i-2} .. phi_{i+3}; plus == 0: the left-biased one, from
 * phi_{i-3} .. phi_{i+2}.  v1..v5 are the five one-sided differences ordered
 * from the far upwind end; three third-order candidates are blended with
 * weights 0.1, 0.6, 0.3 divided by (smoothness + eps)^2.                     */
double oracle_weno5(const double *phi, int64_t n, int64_t i, int plus)
{
    double v[5];
    for (int q = 0; q < 5; ++q) {
        if (plus) {           /* D+ phi_j = phi_{j+1} - phi_j, j = i+2 .. i-2 */
            const int64_t j = i + 2 - q;
            v[q] = phi[wrap(j + 1, n)] - phi[wrap(j, n)];
        } else {              /* D- phi_j = phi_j - phi_{j-1}, j = i-2 .. i+2 */
            const int64_t j = i - 2 + q;
            v[q] = phi[wrap(j, n)] - phi[wrap(j - 1, n)];
        }
    }
    const double p1 = v[0] / 3.0 - 7.0 * v[1] / 6.0 + 11.0 * v[2] / 6.0;
    const double p2 = -v[1] / 6.0 + 5.0 * v[2] / 6.0 + v[3] / 3.0;
    const double p3 = v[2] / 3.0 + 5.0 * v[3] / 6.0 - v[4] / 6.0;
    const double a = v[0] - 2.0 * v[1] + v[2], b = v[0] - 4.0 * v[1] + 3.0 * v[2];
    const double c = v[1] - 2.0 * v[2] + v[3], d = v[1] - v[3];
    const double e = v[2] - 2.0 * v[3] + v[4], g = 3.0 * v[2] - 4.0 * v[3] + v[4];
    const double s1 = 13.0 / 12.0 * a * a + 0.25 * b * b;
    const double s2 = 13.0 / 12.0 * c * c + 0.25 * d * d;
    const double s3 = 13.0 / 12.0 * e * e + 0.25 * g * g;
    double vmax = 0.0;
    for (int q = 0; q < 5; ++q) vmax = fmax(vmax, v[q] * v[q]);
    const double eps = 1e-6 * vmax + 1e-99;
    const double w1 = 0.1 / ((s1 + eps) * (s1 + eps));
    const double w2 = 0.6 / ((s2 + eps) * (s2 + eps));
    const double w3 = 0.3 / ((s3 + eps) * (s3 + eps));
    return (w1 * p1 + w2 * p2 + w3 * p3) / (w1 + w2 + w3);
}

/* One semi-implicit step of the forced Cahn-Hilliard equation in the frame
 * of the travelling wave (the forced flow-pattern section, numerical
 * scheme): the Cahn-Hilliard step above with two more right-hand-side terms,
 * run k having its own parameters,
 *     f_i = C_i + alpha (N_{i-1} - 2 N_i + N_{i+1})
 *           + beta_k W_i(C) + amp_k cos(kdx_k i),
 * W the undivided WENO derivative upwinded for dC/dt = v dC/deta (beta > 0:
 * right-biased, beta < 0: left-biased, beta = 0: no term), with
 * beta = dt v / dx, amp = dt f0 k, kdx = k dx, eta_i = i dx.              */
int oracle_ch_forced_step_batch(int64_t n, int64_t m, int64_t ld, double sigma, double alpha,
                                const double *beta, const double *amp, const double *kdx,
                                const double *c_in, double *c_out)
{
    if (n < 5 || m < 0 || ld < m) return ERR_SIZE;
    double *band = (double *)malloc(sizeof(double) * (size_t)n * 5);
    double *ba = band, *bb = band + n, *bc = band + 2 * n, *bd = band + 3 * n, *be = band + 4 * n;
    for (int64_t i = 0; i < n; ++i) {
        ba[i] = sigma; bb[i] = -4.0 * sigma; bc[i] = 1.0 + 6.0 * sigma;
        bd[i] = -4.0 * sigma; be[i] = sigma;
    }
    int status = OK;
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (size_t)n * 18);
        double *nl = col + n, *f = col + 2 * n, *sol = col + 3 * n, *work = col + 4 * n;
        int my = OK;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            for (int64_t i = 0; i < n; ++i) {
                col[i] = c_in[i * ld + k];
                nl[i] = col[i] * col[i] * col[i] - col[i];
            }
            for (int64_t i = 0; i < n; ++i) {
                double r = col[i] + alpha * (nl[wrap(i - 1, n)] - 2.0 * nl[i] + nl[wrap(i + 1, n)]);
                if (beta[k] != 0.0) r += beta[k] * oracle_weno5(col, n, i, beta[k] > 0.0);
                r += amp[k] * cos(kdx[k] * (double)i);
                f[i] = r;
            }
            int s = oracle_penta_cyclic_solve(n, ba, bb, bc, bd, be, f, sol, work);
            if (s && !my) my = s;
            for (int64_t i = 0; i < n; ++i) c_out[i * ld + k] = s ? NAN : sol[i];
        }
        free(col);
#pragma omp critical
        { if (my && !status) status = my; }
    }
    free(band);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Crank-Nicolson time steps of the benchmark problems: periodic diffusion
 * (Section 3, benchmark problem: LHS bands -s, 1+2s, -s; right-hand side
 * s C_{i-1} + (1-2s) C_i + s C_{i+1}, s = dt/(2 dx^2)) and periodic
 * hyperdiffusion (Section 4, benchmark problem: LHS bands s, -4s, 1+6s, -4s, s;
 * right-hand side -s, 4s, 1-6s, 4s, -s, s = dt/(2 dx^4)).  One step is
 *     A C^{n+1} = B C^n,   (B C)_i = sum_{d=-K..K} w[d+K] C_{i+d},
 * with K = 1 (tri, kind 0/1) or 2 (penta, kind 2/3).  Cyclic kinds wrap the
 * indices of B mod n like the matrix; the others leave out the terms whose
 * index falls outside 0..n-1 (zero boundary values).  The solve is the
 * per-system solver of oracle_solve_batch.                                 */
int oracle_cn_step_batch(int kind, int64_t n, int64_t m, int64_t ld, const double *a,
                         const double *b, const double *c, const double *d, const double *e,
                         const double *w, const double *c_in, double *c_out)
{
    if (n < 1 || m < 0 || ld < m || kind < 0 || kind > 3) return ERR_SIZE;
    const int K = (kind < 2) ? 1 : 2;
    const int cyclic = (kind == 1 || kind == 3);
    int status = OK;
#pragma omp parallel
    {
        double *col = (double *)malloc(sizeof(double) * (size_t)n * 17);
        double *f = col + n, *sol = col + 2 * n, *work = col + 3 * n;   /* 14n of workspace */
        int my = OK;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            for (int64_t i = 0; i < n; ++i) col[i] = c_in[i * ld + k];
            for (int64_t i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int dd = -K; dd <= K; ++dd) {
                    int64_t r = i + dd;
                    if (r < 0 || r >= n) {
                        if (!cyclic) continue;
                        r = wrap(r, n);
                    }
                    acc += w[dd + K] * col[r];
                }
                f[i] = acc;
            }
            int s;
            switch (kind) {
            case 0: s = oracle_tri_solve(n, a, b, c, f, sol, work); break;
            case 1: s = oracle_tri_cyclic_solve(n, a, b, c, f, sol, work); break;
            case 2: s = oracle_penta_solve(n, a, b, c, d, e, f, sol, work); break;
            default: s = oracle_penta_cyclic_solve(n, a, b, c, d, e, f, sol, work); break;
            }
            if (s && !my) my = s;
            for (int64_t i = 0; i < n; ++i) c_out[i * ld + k] = s ? NAN : sol[i];
        }
        free(col);
#pragma omp critical
        { if (my && !status) status = my; }
    }
    return status;
}

/* number of OpenMP threads a parallel region gets (for reporting) */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
#else
int oracle_num_threads(void) { return 1; }
#endif
