// factor.cpp -- host factorisation of the shared matrix and the coefficient
// tables the gfx950 sweep kernels read.  Double precision throughout.
#include "factor.h"

#include <cmath>
#include <string>

namespace bb {

namespace {

bool bad(double p) { return p == 0.0 || !std::isfinite(p); }

std::string at_row(const char *what, int64_t i)
{
    return std::string(what) + " at row " + std::to_string(i);
}

// Tridiagonal LU (Thomas pre-factorisation, Section 3.1; Appendix A):
// b^_0 = b_0, c^_i = c_i / b^_i, b^_i = b_i - a_i c^_{i-1}.  The forward sweep
// d^_i = (d_i - a_i d^_{i-1}) / b^_i and backward sweep x_i = d^_i - c^_i x_{i+1}
// become, with reciprocals stored:
//   primal:  s = 1/b^_i, l1 = a_i/b^_i, u1 = c^_i
//   adjoint (A^T = U^T L^T, rescaled so the backward step has unit diagonal):
//            s = 1/b^_i, l1 = c_{i-1}/b^_i, u1 = a_{i+1}/b^_i
int factor_tri(const double *a, const double *b, const double *c, int64_t n, Recurrence &pr,
               Recurrence &ad, std::vector<double> *bhat_out, std::string &err)
{
    std::vector<double> bhat(n), chat(n);
    for (int64_t i = 0; i < n; ++i) {
        const double ai = i > 0 ? a[i] : 0.0;
        bhat[i] = b[i] - (i > 0 ? ai * chat[i - 1] : 0.0);
        if (bad(bhat[i])) { err = at_row("zero or non-finite pivot b^", i); return kErrPivot; }
        chat[i] = i < n - 1 ? c[i] / bhat[i] : 0.0;
    }
    pr.s.resize(n); pr.l1.resize(n); pr.u1.resize(n);
    ad.s.resize(n); ad.l1.resize(n); ad.u1.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        const double r = 1.0 / bhat[i];
        pr.s[i] = r;
        pr.l1[i] = i > 0 ? a[i] * r : 0.0;
        pr.u1[i] = chat[i];
        ad.s[i] = r;
        ad.l1[i] = i > 0 ? c[i - 1] * r : 0.0;
        ad.u1[i] = i < n - 1 ? a[i + 1] * r : 0.0;
    }
    if (bhat_out) *bhat_out = bhat;
    return kOk;
}

// Pentadiagonal LR factorisation (Section 4.1, steps 1-14 written as one loop
// with entries outside the matrix taken as zero):
//   beta_i = b_i - a_i gamma_{i-2},  alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1},
//   gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i,  delta_i = e_i / alpha_i,  eps_i = a_i.
//   primal:  s = 1/alpha_i, l1 = beta_i/alpha_i, l2 = eps_i/alpha_i, u1 = gamma_i, u2 = delta_i
//   adjoint (A^T = R^T L^T, rescaled by alpha):
//            s = 1/alpha_i, l1 = gamma_{i-1} alpha_{i-1}/alpha_i, l2 = delta_{i-2} alpha_{i-2}/alpha_i,
//            u1 = beta_{i+1}/alpha_i, u2 = eps_{i+2}/alpha_i
int factor_penta(const double *a, const double *b, const double *c, const double *d,
                 const double *e, int64_t n, Recurrence &pr, Recurrence &ad, std::string &err)
{
    std::vector<double> al(n), be(n), ga(n), de(n), ep(n);
    for (int64_t i = 0; i < n; ++i) {
        const double ai = i >= 2 ? a[i] : 0.0;
        const double bi = i >= 1 ? b[i] : 0.0;
        const double di = i + 1 < n ? d[i] : 0.0;
        const double ei = i + 2 < n ? e[i] : 0.0;
        const double g2 = i >= 2 ? ga[i - 2] : 0.0, g1 = i >= 1 ? ga[i - 1] : 0.0;
        const double d2 = i >= 2 ? de[i - 2] : 0.0, d1 = i >= 1 ? de[i - 1] : 0.0;
        ep[i] = ai;
        be[i] = bi - ai * g2;
        al[i] = c[i] - ai * d2 - be[i] * g1;
        if (bad(al[i])) { err = at_row("zero or non-finite pivot alpha", i); return kErrPivot; }
        ga[i] = (di - be[i] * d1) / al[i];
        de[i] = ei / al[i];
    }
    for (Recurrence *r : {&pr, &ad}) {
        r->s.resize(n); r->l1.resize(n); r->l2.resize(n); r->u1.resize(n); r->u2.resize(n);
    }
    for (int64_t i = 0; i < n; ++i) {
        const double r = 1.0 / al[i];
        pr.s[i] = r;
        pr.l1[i] = be[i] * r;
        pr.l2[i] = ep[i] * r;
        pr.u1[i] = ga[i];
        pr.u2[i] = de[i];
        ad.s[i] = r;
        ad.l1[i] = i >= 1 ? ga[i - 1] * al[i - 1] * r : 0.0;
        ad.l2[i] = i >= 2 ? de[i - 2] * al[i - 2] * r : 0.0;
        ad.u1[i] = i + 1 < n ? be[i + 1] * r : 0.0;
        ad.u2[i] = i + 2 < n ? ep[i + 2] * r : 0.0;
    }
    return kOk;
}

// One host solve with a recurrence (used only to precompute correction vectors).
std::vector<double> host_solve(const Recurrence &r, int K, const std::vector<double> &f)
{
    const int64_t n = (int64_t)f.size();
    std::vector<double> y(n);
    for (int64_t i = 0; i < n; ++i) {
        double v = r.s[i] * f[i];
        if (i >= 1) v -= r.l1[i] * y[i - 1];
        if (K == 2 && i >= 2) v -= r.l2[i] * y[i - 2];
        y[i] = v;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double v = y[i];
        if (i + 1 < n) v -= r.u1[i] * y[i + 1];
        if (K == 2 && i + 2 < n) v -= r.u2[i] * y[i + 2];
        y[i] = v;
    }
    return y;
}

// A capacitance (1 + V.z, or det(I + V^T Z)) that cancels to rounding level
// means the periodic matrix is numerically singular.
bool negligible(double value, double scale)
{
    return bad(value) || std::fabs(value) <= 1024.0 * 2.220446049250313e-16 * scale;
}

bool inv2(const double m[4], double out[4])
{
    const double det = m[0] * m[3] - m[1] * m[2];
    if (negligible(det, std::fabs(m[0] * m[3]) + std::fabs(m[1] * m[2]))) return false;
    out[0] = m[3] / det; out[1] = -m[1] / det;
    out[2] = -m[2] / det; out[3] = m[0] / det;
    return true;
}

}  // namespace

Factor::~Factor()
{
    for (auto &kv : dev) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    for (auto &kv : dev_paper) if (kv.second.ptr) (void)hipFree(kv.second.ptr);
}

int make_factor_impl(int kind, const double *const bands[5], int64_t n, Factor &f, std::string &err);

int make_factor(int kind, const double *const bands[5], int64_t n, Factor &f, std::string &err)
{
    const int st = make_factor_impl(kind, bands, n, f, err);
    if (st == kOk && f.n >= 2) {
        // -u1 of row n-2 of each direction (the table stores u1 negated)
        f.primal.cor.q.u1_nm2 = -f.primal.rec.u1[f.n - 2];
        f.adjoint.cor.q.u1_nm2 = -f.adjoint.rec.u1[f.n - 2];
    }
    return st;
}

int make_factor_impl(int kind, const double *const bands[5], int64_t n, Factor &f, std::string &err)
{
    f.kind = kind;
    f.K = (kind == kTri || kind == kTriCyclic) ? 1 : 2;
    f.cyclic = (kind == kTriCyclic || kind == kPentaCyclic);
    f.n = n;
    const int K = f.K;
    const int nb = 2 * K + 1;
    for (int q = 0; q < nb; ++q) f.band[q].assign(bands[q], bands[q] + n);
    // zero the entries that fall outside the matrix (corners go to f.corners)
    for (int q = 0; q < nb; ++q) {
        const int off = q - K;
        for (int64_t i = 0; i < n; ++i)
            if (i + off < 0 || i + off >= n) f.band[q][i] = 0.0;
    }

    if (kind == kTri) {
        int st = factor_tri(bands[0], bands[1], bands[2], n, f.primal.rec, f.adjoint.rec, nullptr, err);
        if (st) return st;
        f.rhat = f.primal.rec.s;
        f.aprime = f.primal.rec.l1;
        f.chat = f.primal.rec.u1;
        return kOk;
    }
    if (kind == kPenta)
        return factor_penta(bands[0], bands[1], bands[2], bands[3], bands[4], n, f.primal.rec,
                            f.adjoint.rec, err);

    if (kind == kTriCyclic) {
        // Section 3.3, generalised to row-dependent bands: U = (-b_0, 0.., c_{n-1}),
        // V = (1, 0.., -a_0/b_0); A' has 2 b_0 and b_{n-1} + a_0 c_{n-1}/b_0 on its diagonal ends.
        const double *a = bands[0], *b = bands[1], *c = bands[2];
        if (bad(b[0])) { err = "zero or non-finite b_0 (cyclic split)"; return kErrPivot; }
        const double aw = a[0], cw = c[n - 1], vlast = -aw / b[0];
        std::vector<double> bp(b, b + n);
        bp[0] = 2.0 * b[0];
        bp[n - 1] = b[n - 1] + aw * cw / b[0];
        int st = factor_tri(a, bp.data(), c, n, f.primal.rec, f.adjoint.rec, nullptr, err);
        if (st) return st;
        f.corners.top[0][1] = aw;
        f.corners.bot[1][0] = cw;
        std::vector<double> U(n, 0.0), V(n, 0.0);
        U[0] = -b[0]; U[n - 1] = cw;
        V[0] = 1.0;  V[n - 1] = vlast;
        // primal: z = A'^{-1} U, s = (V.y) / (1 + V.z)
        std::vector<double> z = host_solve(f.primal.rec, 1, U);
        const double den = 1.0 + z[0] + vlast * z[n - 1];
        if (negligible(den, 1.0 + std::fabs(z[0]) + std::fabs(vlast * z[n - 1]))) { err = "1 + V.z is singular"; return kErrCapacitance; }
        f.primal.cor.z0 = z;
        f.primal.cor.q.q[0][0] = 1.0 / den;
        f.primal.cor.q.q[0][1] = vlast / den;
        // adjoint: A^T = A'^T + V U^T, z' = A'^{-T} V, s = (U.y) / (1 + U.z')
        std::vector<double> zt = host_solve(f.adjoint.rec, 1, V);
        const double dent = 1.0 + U[0] * zt[0] + U[n - 1] * zt[n - 1];
        if (negligible(dent, 1.0 + std::fabs(U[0] * zt[0]) + std::fabs(U[n - 1] * zt[n - 1]))) { err = "1 + U.z' is singular"; return kErrCapacitance; }
        f.adjoint.cor.z0 = zt;
        f.adjoint.cor.q.q[0][0] = U[0] / dent;
        f.adjoint.cor.q.q[0][1] = U[n - 1] / dent;
        return kOk;
    }

    // kPentaCyclic: rank-2 split of the periodic pentadiagonal matrix.
    //   T = A[0:2,0:2], B = A[0:2,n-2:n], Cb = A[n-2:n,0:2], W = T^{-1} B,
    //   U = [-T; 0; Cb], V^T = [I, 0, -W], A' = A - U V^T (top-left 2T,
    //   bottom-right A_BR + Cb W, no corners).
    const double *a = bands[0], *b = bands[1], *c = bands[2], *d = bands[3], *e = bands[4];
    const double T[4] = {c[0], d[0], b[1], c[1]};
    const double B[4] = {a[0], b[0], 0.0, a[1]};
    const double Cb[4] = {e[n - 2], 0.0, d[n - 1], e[n - 1]};
    double Ti[4];
    if (!inv2(T, Ti)) { err = "top-left 2x2 block is singular (cyclic split)"; return kErrPivot; }
    const double W[4] = {Ti[0] * B[0] + Ti[1] * B[2], Ti[0] * B[1] + Ti[1] * B[3],
                         Ti[2] * B[0] + Ti[3] * B[2], Ti[2] * B[1] + Ti[3] * B[3]};
    const double CW[4] = {Cb[0] * W[0] + Cb[1] * W[2], Cb[0] * W[1] + Cb[1] * W[3],
                          Cb[2] * W[0] + Cb[3] * W[2], Cb[2] * W[1] + Cb[3] * W[3]};
    std::vector<double> pa(a, a + n), pb(b, b + n), pc(c, c + n), pd(d, d + n), pe(e, e + n);
    pc[0] = 2.0 * T[0]; pd[0] = 2.0 * T[1]; pb[1] = 2.0 * T[2]; pc[1] = 2.0 * T[3];
    pc[n - 2] = c[n - 2] + CW[0]; pd[n - 2] = d[n - 2] + CW[1];
    pb[n - 1] = b[n - 1] + CW[2]; pc[n - 1] = c[n - 1] + CW[3];
    int st = factor_penta(pa.data(), pb.data(), pc.data(), pd.data(), pe.data(), n, f.primal.rec,
                          f.adjoint.rec, err);
    if (st) return st;
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) {
            f.corners.top[r][q] = B[r * 2 + q];
            f.corners.bot[r][q] = Cb[r * 2 + q];
        }
    // primal: Z = A'^{-1} U, H = (I + V^T Z)^{-1}, s = H (y_top - W y_bot)
    std::vector<double> u0(n, 0.0), u1(n, 0.0);
    u0[0] = -T[0]; u1[0] = -T[1];
    u0[1] = -T[2]; u1[1] = -T[3];
    u0[n - 2] = Cb[0]; u1[n - 2] = Cb[1];
    u0[n - 1] = Cb[2]; u1[n - 1] = Cb[3];
    std::vector<double> z0 = host_solve(f.primal.rec, 2, u0), z1 = host_solve(f.primal.rec, 2, u1);
    auto vt = [&](const std::vector<double> &y, int r) {   // (V^T y)_r
        return y[r] - (W[r * 2 + 0] * y[n - 2] + W[r * 2 + 1] * y[n - 1]);
    };
    const double IVZ[4] = {1.0 + vt(z0, 0), vt(z1, 0), vt(z0, 1), 1.0 + vt(z1, 1)};
    double H[4];
    if (!inv2(IVZ, H)) { err = "I + V^T Z is singular"; return kErrCapacitance; }
    f.primal.cor.z0 = z0;
    f.primal.cor.z1 = z1;
    // s = H [y0, y1]^T - H W [y_{n-2}, y_{n-1}]^T  ->  Q = [H, -H W]
    const double HW[4] = {H[0] * W[0] + H[1] * W[2], H[0] * W[1] + H[1] * W[3],
                          H[2] * W[0] + H[3] * W[2], H[2] * W[1] + H[3] * W[3]};
    for (int r = 0; r < 2; ++r) {
        f.primal.cor.q.q[r][0] = H[r * 2 + 0];
        f.primal.cor.q.q[r][1] = H[r * 2 + 1];
        f.primal.cor.q.q[r][2] = -HW[r * 2 + 0];
        f.primal.cor.q.q[r][3] = -HW[r * 2 + 1];
    }
    // adjoint: A^T = A'^T + V U^T, Z' = A'^{-T} V, H' = (I + U^T Z')^{-1},
    // s = H' U^T y with U^T y = -T^T y_top + Cb^T y_bot
    std::vector<double> v0(n, 0.0), v1(n, 0.0);   // columns of V = [I; 0; -W^T]
    v0[0] = 1.0; v1[1] = 1.0;
    v0[n - 2] = -W[0]; v0[n - 1] = -W[1];
    v1[n - 2] = -W[2]; v1[n - 1] = -W[3];
    std::vector<double> w0 = host_solve(f.adjoint.rec, 2, v0), w1 = host_solve(f.adjoint.rec, 2, v1);
    // (U^T y)_r = -(T[0][r] y0 + T[1][r] y1) + Cb[0][r] y_{n-2} + Cb[1][r] y_{n-1}
    auto ut = [&](const std::vector<double> &y, int r) {
        return -(T[0 * 2 + r] * y[0] + T[1 * 2 + r] * y[1]) + Cb[0 * 2 + r] * y[n - 2] +
               Cb[1 * 2 + r] * y[n - 1];
    };
    const double IUZ[4] = {1.0 + ut(w0, 0), ut(w1, 0), ut(w0, 1), 1.0 + ut(w1, 1)};
    double Hp[4];
    if (!inv2(IUZ, Hp)) { err = "I + U^T Z' is singular"; return kErrCapacitance; }
    f.adjoint.cor.z0 = w0;
    f.adjoint.cor.z1 = w1;
    // Q' = H' [-T^T, Cb^T]
    for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) {
            // (H' (-T^T))[r][q] = -sum_p H'[r][p] T[q][p]
            f.adjoint.cor.q.q[r][q] = -(Hp[r * 2 + 0] * T[q * 2 + 0] + Hp[r * 2 + 1] * T[q * 2 + 1]);
            // (H' Cb^T)[r][q] = sum_p H'[r][p] Cb[q][p]
            f.adjoint.cor.q.q[r][2 + q] = Hp[r * 2 + 0] * Cb[q * 2 + 0] + Hp[r * 2 + 1] * Cb[q * 2 + 1];
        }
    return kOk;
}

int choose_chunk(int64_t n, int cmax)
{
    if (cmax > kChunkMax) cmax = kChunkMax;
    if (cmax < kChunkMin) cmax = kChunkMin;
    const int P = lanes_for(n, cmax);
    int C = kChunkMin;
    while ((int64_t)C * P < n) C *= 2;
    return C;
}

int lanes_for(int64_t n, int C)
{
    int P = 1;
    while ((int64_t)P * C < n && P < kWave) P *= 2;
    return P;
}

std::vector<double> build_table(const Direction &d, int K, bool cyclic, int64_t n, int C, int P)
{
    const int64_t L = (int64_t)P * (C + 1);
    const int na = num_arrays(K, cyclic);
    std::vector<double> tab((size_t)table_len(K, cyclic, C, P), 0.0);
    const Recurrence &r = d.rec;
    auto coef = [&](const std::vector<double> &v, int64_t row) {
        return row < n && !v.empty() ? v[row] : 0.0;
    };
    auto at = [&](int q, int j, int t) -> double & {
        return tab[(size_t)(q * L + (int64_t)j * (C + 1) + t)];
    };
    // array indices of the layout in internal.h
    const int qE = 0, qS = K, qs = 2 * K, ql = 2 * K + 1, qu = 3 * K + 1, qz = 4 * K + 1;
    double *Mf = tab.data() + na * L;
    double *Mb = Mf + (int64_t)P * K * K;
    double *G = Mb + (int64_t)P * K * K;

    std::vector<double> y(C), x(C);
    for (int j = 0; j < P; ++j) {
        const int64_t r0 = (int64_t)j * C;
        // forward recurrence over the chunk for right-hand side f (C values) and
        // history (h1, h2); backward recurrence for input y and future (g1, g2)
        auto forward = [&](const double *f, double h1, double h2) {
            for (int t = 0; t < C; ++t) {
                const int64_t row = r0 + t;
                double v = (f ? coef(r.s, row) * f[t] : 0.0) - coef(r.l1, row) * h1;
                if (K == 2) v -= coef(r.l2, row) * h2;
                y[t] = v;
                h2 = h1;
                h1 = v;
            }
        };
        auto backward = [&](const std::vector<double> &in, double g1, double g2) {
            for (int t = C - 1; t >= 0; --t) {
                const int64_t row = r0 + t;
                double v = in[t] - coef(r.u1, row) * g1;
                if (K == 2) v -= coef(r.u2, row) * g2;
                x[t] = v;
                g2 = g1;
                g1 = v;
            }
        };
        // weights of e and o: responses to a unit right-hand side at each row
        std::vector<double> unit(C, 0.0);
        for (int tau = 0; tau < C; ++tau) {
            unit.assign(C, 0.0);
            unit[tau] = 1.0;
            forward(unit.data(), 0.0, 0.0);
            at(qE, j, tau) = y[C - 1];
            if (K == 2) at(qE + 1, j, tau) = y[C - 2];
            backward(y, 0.0, 0.0);
            at(qS, j, tau) = x[0];
            if (K == 2) at(qS + 1, j, tau) = x[1];
        }
        for (int comp = 0; comp < K; ++comp) {
            // history unit vector: end state (Mf) and backward start state (G)
            forward(nullptr, comp == 0 ? 1.0 : 0.0, comp == 1 ? 1.0 : 0.0);
            Mf[j * K * K + 0 * K + comp] = y[C - 1];
            if (K == 2) Mf[j * K * K + 1 * K + comp] = y[C - 2];
            backward(y, 0.0, 0.0);
            G[j * K * K + 0 * K + comp] = x[0];
            if (K == 2) G[j * K * K + 1 * K + comp] = x[1];
            // future unit vector: start state (Mb)
            std::vector<double> zero(C, 0.0);
            backward(zero, comp == 0 ? 1.0 : 0.0, comp == 1 ? 1.0 : 0.0);
            Mb[j * K * K + 0 * K + comp] = x[0];
            if (K == 2) Mb[j * K * K + 1 * K + comp] = x[1];
        }
        // recurrence coefficients (off-diagonal ones and z negated: one fma per step)
        for (int t = 0; t < C; ++t) {
            const int64_t row = r0 + t;
            if (row >= n) continue;
            at(qs, j, t) = r.s[row];
            at(ql, j, t) = -r.l1[row];
            if (K == 2) at(ql + 1, j, t) = -r.l2[row];
            at(qu, j, t) = -r.u1[row];
            if (K == 2) at(qu + 1, j, t) = -r.u2[row];
            if (cyclic) {
                at(qz, j, t) = -d.cor.z0[row];
                if (K == 2) at(qz + 1, j, t) = -d.cor.z1[row];
            }
        }
    }
    return tab;
}

std::vector<double> build_band_table(const Factor &f, int C, int P)
{
    const int64_t L = (int64_t)P * (C + 1);
    const int nb = 2 * f.K + 1;
    std::vector<double> tab((size_t)(nb * L), 0.0);
    for (int q = 0; q < nb; ++q)
        for (int j = 0; j < P; ++j)
            for (int t = 0; t < C; ++t) {
                const int64_t row = (int64_t)j * C + t;
                if (row < f.n) tab[(size_t)(q * L + (int64_t)j * (C + 1) + t)] = f.band[q][row];
            }
    return tab;
}

}  // namespace bb
