// chunk_emu.cpp -- CPU model of the GPU sweep's dataflow, for tests only.
//
// Builds the library's host factor and coefficient table (factor.cpp, the
// product code) and replays, lane by lane in double, exactly what one wave
// does for one system: the boundary-state dot products, the two scans over
// chunks, the forward and backward passes and the periodic correction.  A
// CPU test compares the result with the oracle, so the table construction
// and the decomposition are checked without a GPU.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2107_05395_amd/csrc/factor.h"

extern "C" int emu_solve(int kind, const double *a, const double *b, const double *c,
                         const double *d, const double *e, int64_t n, int adjoint, int C,
                         const double *f, double *x)
{
    bb::Factor F;
    std::string err;
    const double *bands[5] = {a, b, c, d, e};
    int st = bb::make_factor(kind, bands, n, F, err);
    if (st) return st;
    const int K = F.K;
    const int P = bb::lanes_for(n, C);
    if ((int64_t)P * C < n) return -100;
    const bb::Direction &dir = adjoint ? F.adjoint : F.primal;
    const std::vector<double> tab = bb::build_table(dir, K, F.cyclic, n, C, P);
    const int64_t L = (int64_t)P * (C + 1);
    const int na = bb::num_arrays(K, F.cyclic);
    auto arr = [&](int q, int j, int t) { return tab[(size_t)(q * L + (int64_t)j * (C + 1) + t)]; };
    const double *Mf = tab.data() + na * L, *Mb = Mf + P * K * K, *G = Mb + P * K * K;
    const int qE = 0, qS = K, qs = 2 * K, ql = 2 * K + 1, qu = 3 * K + 1, qz = 4 * K + 1;

    std::vector<std::vector<double>> v(P, std::vector<double>(C, 0.0));
    for (int j = 0; j < P; ++j)
        for (int t = 0; t < C; ++t) v[j][t] = j * C + t < n ? f[j * C + t] : 0.0;
    // pass 1
    std::vector<double> e1(P, 0), e2(P, 0), o1(P, 0), o2(P, 0);
    for (int j = 0; j < P; ++j)
        for (int t = 0; t < C; ++t) {
            e1[j] += arr(qE, j, t) * v[j][t];
            o1[j] += arr(qS, j, t) * v[j][t];
            if (K == 2) {
                e2[j] += arr(qE + 1, j, t) * v[j][t];
                o2[j] += arr(qS + 1, j, t) * v[j][t];
            }
        }
    auto affine = [&](const double *M, double &y1, double &y2, double a1, double a2) {
        if (K == 1) {
            y1 = M[0] * y1 + a1;
        } else {
            const double n1 = M[0] * y1 + M[1] * y2 + a1, n2 = M[2] * y1 + M[3] * y2 + a2;
            y1 = n1;
            y2 = n2;
        }
    };
    std::vector<double> h1(P, 0), h2(P, 0), s1(P), s2(P), f1(P, 0), f2(P, 0);
    for (int j = 0; j < P; ++j)
        for (int i = 0; i < j; ++i) affine(Mf + i * K * K, h1[j], h2[j], e1[i], e2[i]);
    for (int j = 0; j < P; ++j) {
        const double *g = G + j * K * K;
        s1[j] = o1[j] + g[0] * h1[j] + (K == 2 ? g[1] * h2[j] : 0.0);
        s2[j] = K == 2 ? o2[j] + g[2] * h1[j] + g[3] * h2[j] : 0.0;
    }
    for (int j = 0; j < P; ++j)
        for (int i = P - 1; i > j; --i) affine(Mb + i * K * K, f1[j], f2[j], s1[i], s2[i]);
    // pass 2 and pass 3 (correction applied afterwards, from the solution ends)
    for (int j = 0; j < P; ++j) {
        double y1 = h1[j], y2 = h2[j];
        for (int t = 0; t < C; ++t) {
            double y = arr(qs, j, t) * v[j][t];
            if (K == 2) y += arr(ql + 1, j, t) * y2;
            y += arr(ql, j, t) * y1;
            v[j][t] = y;
            y2 = y1;
            y1 = y;
        }
        double x1 = f1[j], x2 = f2[j];
        for (int t = C - 1; t >= 0; --t) {
            double xx = v[j][t];
            if (K == 2) xx += arr(qu + 1, j, t) * x2;
            xx += arr(qu, j, t) * x1;
            v[j][t] = xx;
            x2 = x1;
            x1 = xx;
        }
    }
    if (F.cyclic) {
        const bb::CyclicQ &q = dir.cor.q;
        auto at = [&](int64_t row) { return v[row / C][row % C]; };
        double c0, c1 = 0.0;
        if (K == 1) {
            c0 = q.q[0][0] * at(0) + q.q[0][1] * at(n - 1);
        } else {
            const double r[4] = {at(0), at(1), at(n - 2), at(n - 1)};
            c0 = q.q[0][0] * r[0] + q.q[0][1] * r[1] + q.q[0][2] * r[2] + q.q[0][3] * r[3];
            c1 = q.q[1][0] * r[0] + q.q[1][1] * r[1] + q.q[1][2] * r[2] + q.q[1][3] * r[3];
        }
        // cross-check the fused form the kernel uses when chunks tile n exactly
        if (n % C == 0) {
            const int jl = (int)(n / C) - 1;
            double x0 = f1[0], x1v = f2[0];
            affine(Mb, x0, x1v, s1[0], s2[0]);
            double y1 = h1[jl], y2 = h2[jl];
            affine(Mf + jl * K * K, y1, y2, e1[jl], e2[jl]);
            const double rn1 = y1, rn2 = K == 2 ? q.u1_nm2 * rn1 + y2 : 0.0;
            double d0, d1 = 0.0;
            if (K == 1) {
                d0 = q.q[0][0] * x0 + q.q[0][1] * rn1;
            } else {
                d0 = q.q[0][0] * x0 + q.q[0][1] * x1v + q.q[0][2] * rn2 + q.q[0][3] * rn1;
                d1 = q.q[1][0] * x0 + q.q[1][1] * x1v + q.q[1][2] * rn2 + q.q[1][3] * rn1;
            }
            const double tol = 1e-9 * (1.0 + std::abs(c0) + std::abs(c1));
            if (std::abs(d0 - c0) > tol || std::abs(d1 - c1) > tol) return -101;
        }
        for (int j = 0; j < P; ++j)
            for (int t = 0; t < C; ++t)
                v[j][t] += arr(qz, j, t) * c0 + (K == 2 ? arr(qz + 1, j, t) * c1 : 0.0);
    }
    for (int64_t i = 0; i < n; ++i) x[i] = v[i / C][i % C];
    return 0;
}

// The three-launch decomposition of long systems (long_core.h), replayed for
// one system in double: the solution array x doubles as the scratch of the
// launches exactly as on the device (e, o, then H, F and the periodic
// correction scalars in the first 3K rows of every full chunk).
extern "C" int emu_solve_long(int kind, const double *a, const double *b, const double *c,
                              const double *d, const double *e, int64_t n, int adjoint, int C,
                              const double *f, double *x)
{
    bb::Factor F;
    std::string err;
    const double *bands[5] = {a, b, c, d, e};
    int st = bb::make_factor(kind, bands, n, F, err);
    if (st) return st;
    const int K = F.K;
    const int P = (int)((n + C - 1) / C);
    if (P < 2 || C < 3 * K) return -100;
    const int full = P - 1;
    const bb::Direction &dir = adjoint ? F.adjoint : F.primal;
    const std::vector<double> tab = bb::build_table(dir, K, F.cyclic, n, C, P);
    const int64_t L = (int64_t)P * (C + 1);
    const int na = bb::num_arrays(K, F.cyclic);
    auto arr = [&](int q, int j, int t) { return tab[(size_t)(q * L + (int64_t)j * (C + 1) + t)]; };
    const double *Mf = tab.data() + na * L, *Mb = Mf + P * K * K, *G = Mb + P * K * K;
    const int qE = 0, qS = K, qs = 2 * K, ql = 2 * K + 1, qu = 3 * K + 1, qz = 4 * K + 1;
    auto affine = [&](const double *M, double &y1, double &y2, double a1, double a2) {
        if (K == 1) {
            y1 = M[0] * y1 + a1;
        } else {
            const double n1 = M[0] * y1 + M[1] * y2 + a1, n2 = M[2] * y1 + M[3] * y2 + a2;
            y1 = n1;
            y2 = n2;
        }
    };
    auto fwd = [&](std::vector<double> &v, int j, double h1, double h2) {
        for (int t = 0; t < C; ++t) {
            double y = arr(qs, j, t) * v[t];
            if (K == 2) y += arr(ql + 1, j, t) * h2;
            y += arr(ql, j, t) * h1;
            v[t] = y;
            h2 = h1;
            h1 = y;
        }
    };
    auto bwd = [&](std::vector<double> &v, int j, double g1, double g2, double c0, double c1) {
        for (int t = C - 1; t >= 0; --t) {
            double xx = v[t];
            if (K == 2) xx += arr(qu + 1, j, t) * g2;
            xx += arr(qu, j, t) * g1;
            g2 = g1;
            g1 = xx;
            if (F.cyclic) xx += arr(qz, j, t) * c0 + (K == 2 ? arr(qz + 1, j, t) * c1 : 0.0);
            v[t] = xx;
        }
    };
    // reduce
    for (int j = 0; j < full; ++j) {
        double e1 = 0, e2 = 0, o1 = 0, o2 = 0;
        for (int t = 0; t < C; ++t) {
            const double v = f[j * C + t];
            e1 += arr(qE, j, t) * v;
            o1 += arr(qS, j, t) * v;
            if (K == 2) {
                e2 += arr(qE + 1, j, t) * v;
                o2 += arr(qS + 1, j, t) * v;
            }
        }
        x[j * C] = e1;
        if (K == 2) x[j * C + 1] = e2;
        x[j * C + K] = o1;
        if (K == 2) x[j * C + K + 1] = o2;
    }
    // scan
    double h1 = 0, h2 = 0;
    for (int j = 0; j < full; ++j) {
        const double a1 = x[j * C], a2 = K == 2 ? x[j * C + 1] : 0.0;
        x[j * C] = h1;
        if (K == 2) x[j * C + 1] = h2;
        affine(Mf + j * K * K, h1, h2, a1, a2);
    }
    const int64_t tr0 = (int64_t)full * C;
    const int nr = (int)(n - tr0);
    std::vector<double> v(C, 0.0);
    for (int t = 0; t < nr; ++t) v[t] = f[tr0 + t];
    fwd(v, full, h1, h2);
    const double yn1 = v[nr - 1], yn2 = nr >= 2 ? v[nr - 2] : h1;
    bwd(v, full, 0.0, 0.0, 0.0, 0.0);
    double f1 = v[0], f2 = K == 2 ? v[1] : 0.0;
    for (int j = full - 1; j >= 0; --j) {
        const double *g = G + j * K * K;
        const double hh1 = x[j * C], hh2 = K == 2 ? x[j * C + 1] : 0.0;
        const double s1 = x[j * C + K] + g[0] * hh1 + (K == 2 ? g[1] * hh2 : 0.0);
        const double s2 = K == 2 ? x[j * C + K + 1] + g[2] * hh1 + g[3] * hh2 : 0.0;
        x[j * C + K] = f1;
        if (K == 2) x[j * C + K + 1] = f2;
        affine(Mb + j * K * K, f1, f2, s1, s2);
    }
    double c0 = 0.0, c1 = 0.0;
    if (F.cyclic) {
        const bb::CyclicQ &q = dir.cor.q;
        const double rn1 = yn1, rn2 = K == 2 ? q.u1_nm2 * rn1 + yn2 : 0.0;
        if (K == 1) {
            c0 = q.q[0][0] * f1 + q.q[0][1] * rn1;
        } else {
            c0 = q.q[0][0] * f1 + q.q[0][1] * f2 + q.q[0][2] * rn2 + q.q[0][3] * rn1;
            c1 = q.q[1][0] * f1 + q.q[1][1] * f2 + q.q[1][2] * rn2 + q.q[1][3] * rn1;
        }
        for (int j = 0; j < full; ++j) {
            x[j * C + 2 * K] = c0;
            if (K == 2) x[j * C + 2 * K + 1] = c1;
        }
        for (int t = 0; t < C; ++t)
            v[t] += arr(qz, full, t) * c0 + (K == 2 ? arr(qz + 1, full, t) * c1 : 0.0);
    }
    for (int t = 0; t < nr; ++t) x[tr0 + t] = v[t];
    // solve
    for (int j = 0; j < full; ++j) {
        const double H1 = x[j * C], H2 = K == 2 ? x[j * C + 1] : 0.0;
        const double G1 = x[j * C + K], G2 = K == 2 ? x[j * C + K + 1] : 0.0;
        const double C0 = F.cyclic ? x[j * C + 2 * K] : 0.0;
        const double C1 = F.cyclic && K == 2 ? x[j * C + 2 * K + 1] : 0.0;
        std::vector<double> w(f + j * C, f + (j + 1) * C);
        fwd(w, j, H1, H2);
        bwd(w, j, G1, G2, C0, C1);
        for (int t = 0; t < C; ++t) x[j * C + t] = w[t];
    }
    return 0;
}

// Affine maps y -> c + M y of the chunks, for the small-batch scan of long
// systems below (long_scan_spread); reduce and solve as in emu_solve_long.
namespace {
struct Aff {
    double m[4], c[2];
};
Aff aff_id() { return Aff{{1, 0, 0, 1}, {0, 0}}; }
// r = x after a (apply a first)
Aff aff_after(const Aff &x, const Aff &a, int K)
{
    Aff r;
    if (K == 1) {
        r = aff_id();
        r.c[0] = x.m[0] * a.c[0] + x.c[0];
        r.m[0] = x.m[0] * a.m[0];
        return r;
    }
    r.c[0] = x.m[0] * a.c[0] + x.m[1] * a.c[1] + x.c[0];
    r.c[1] = x.m[2] * a.c[0] + x.m[3] * a.c[1] + x.c[1];
    r.m[0] = x.m[0] * a.m[0] + x.m[1] * a.m[2];
    r.m[1] = x.m[0] * a.m[1] + x.m[1] * a.m[3];
    r.m[2] = x.m[2] * a.m[0] + x.m[3] * a.m[2];
    r.m[3] = x.m[2] * a.m[1] + x.m[3] * a.m[3];
    return r;
}
Aff aff_of(const double *M, double e1, double e2, int K)
{
    Aff t = aff_id();
    t.m[0] = M[0];
    if (K == 2) { t.m[1] = M[1]; t.m[2] = M[2]; t.m[3] = M[3]; }
    t.c[0] = e1;
    t.c[1] = e2;
    return t;
}
}  // namespace

// The small-batch scan of long systems: blocks of 64 full chunks in the
// chain's order (forward from chunk 0, backward from the last full chunk),
// each block's affine maps scanned across the 64 lanes (Hillis-Steele, the
// identity past the block's last chunk), the state entering a chunk being
// the composition up to the previous lane applied to the block's entering
// state.
extern "C" int emu_solve_long_spread(int kind, const double *a, const double *b, const double *c,
                                     const double *d, const double *e, int64_t n, int adjoint,
                                     int C, const double *f, double *x)
{
    bb::Factor F;
    std::string err;
    const double *bands[5] = {a, b, c, d, e};
    int st = bb::make_factor(kind, bands, n, F, err);
    if (st) return st;
    const int K = F.K, W = 64;
    const int P = (int)((n + C - 1) / C);
    const int full = P - 1;
    if (P < 2 || C < 3 * K) return -100;
    const bb::Direction &dir = adjoint ? F.adjoint : F.primal;
    const std::vector<double> tab = bb::build_table(dir, K, F.cyclic, n, C, P);
    const int64_t L = (int64_t)P * (C + 1);
    const int na = bb::num_arrays(K, F.cyclic);
    auto arr = [&](int q, int j, int t) { return tab[(size_t)(q * L + (int64_t)j * (C + 1) + t)]; };
    const double *Mf = tab.data() + na * L, *Mb = Mf + P * K * K, *G = Mb + P * K * K;
    const int qE = 0, qS = K, qs = 2 * K, ql = 2 * K + 1, qu = 3 * K + 1, qz = 4 * K + 1;
    // reduce
    std::vector<double> e1(full), e2(full), o1(full), o2(full);
    for (int j = 0; j < full; ++j) {
        double s1 = 0, s2 = 0, t1 = 0, t2 = 0;
        for (int t = 0; t < C; ++t) {
            const double v = f[j * C + t];
            s1 += arr(qE, j, t) * v;
            t1 += arr(qS, j, t) * v;
            if (K == 2) {
                s2 += arr(qE + 1, j, t) * v;
                t2 += arr(qS + 1, j, t) * v;
            }
        }
        e1[j] = s1; e2[j] = s2; o1[j] = t1; o2[j] = t2;
    }
    // one block: maps[l] for l < cnt, identity beyond; returns the entering
    // state of every lane and advances (y1, y2) past the block
    auto block = [&](std::vector<Aff> maps, int cnt, double &y1, double &y2,
                     std::vector<double> &in1, std::vector<double> &in2) {
        for (int l = cnt; l < W; ++l) maps[l] = aff_id();
        for (int dd = 1; dd < W; dd <<= 1) {
            std::vector<Aff> B = maps;
            for (int l = dd; l < W; ++l) B[l] = aff_after(maps[l], maps[l - dd], K);
            maps = B;
        }
        in1.assign(W, 0.0);
        in2.assign(W, 0.0);
        for (int l = 0; l < W; ++l) {
            const Aff p = l ? maps[l - 1] : aff_id();
            in1[l] = p.m[0] * y1 + (K == 2 ? p.m[1] * y2 : 0.0) + p.c[0];
            in2[l] = K == 2 ? p.m[2] * y1 + p.m[3] * y2 + p.c[1] : 0.0;
        }
        const Aff &t = maps[W - 1];
        const double n1 = t.m[0] * y1 + (K == 2 ? t.m[1] * y2 : 0.0) + t.c[0];
        const double n2 = K == 2 ? t.m[2] * y1 + t.m[3] * y2 + t.c[1] : 0.0;
        y1 = n1; y2 = n2;
    };
    std::vector<double> H1(full), H2(full), in1, in2;
    double h1 = 0.0, h2 = 0.0;
    for (int j0 = 0; j0 < full; j0 += W) {
        const int cnt = std::min(W, full - j0);
        std::vector<Aff> maps(W, aff_id());
        for (int l = 0; l < cnt; ++l) maps[l] = aff_of(Mf + (j0 + l) * K * K, e1[j0 + l], e2[j0 + l], K);
        block(maps, cnt, h1, h2, in1, in2);
        for (int l = 0; l < cnt; ++l) { H1[j0 + l] = in1[l]; H2[j0 + l] = in2[l]; }
    }
    // the tail
    const int64_t tr0 = (int64_t)full * C;
    const int nr = (int)(n - tr0);
    std::vector<double> v(C, 0.0);
    for (int t = 0; t < nr; ++t) v[t] = f[tr0 + t];
    {
        double y1 = h1, y2 = h2;
        for (int t = 0; t < C; ++t) {
            double y = arr(qs, full, t) * v[t];
            if (K == 2) y += arr(ql + 1, full, t) * y2;
            y += arr(ql, full, t) * y1;
            v[t] = y; y2 = y1; y1 = y;
        }
    }
    const double yn1 = v[nr - 1], yn2 = nr >= 2 ? v[nr - 2] : h1;
    {
        double x1 = 0, x2 = 0;
        for (int t = C - 1; t >= 0; --t) {
            double xx = v[t];
            if (K == 2) xx += arr(qu + 1, full, t) * x2;
            xx += arr(qu, full, t) * x1;
            x2 = x1; x1 = xx; v[t] = xx;
        }
    }
    // backward: S_j, blocks from the last full chunk down
    std::vector<double> F1(full), F2(full);
    double f1 = v[0], f2 = K == 2 ? v[1] : 0.0;
    for (int jt = full - 1; jt >= 0; jt -= W) {
        const int cnt = std::min(W, jt + 1);
        std::vector<Aff> maps(W, aff_id());
        for (int l = 0; l < cnt; ++l) {
            const int j = jt - l;
            const double *g = G + j * K * K;
            const double s1 = o1[j] + g[0] * H1[j] + (K == 2 ? g[1] * H2[j] : 0.0);
            const double s2 = K == 2 ? o2[j] + g[2] * H1[j] + g[3] * H2[j] : 0.0;
            maps[l] = aff_of(Mb + j * K * K, s1, s2, K);
        }
        block(maps, cnt, f1, f2, in1, in2);
        for (int l = 0; l < cnt; ++l) { F1[jt - l] = in1[l]; F2[jt - l] = in2[l]; }
    }
    const double w0 = f1, w1 = f2;
    double c0 = 0, c1 = 0;
    if (F.cyclic) {
        const bb::CyclicQ &q = dir.cor.q;
        const double rn1 = yn1, rn2 = K == 2 ? q.u1_nm2 * rn1 + yn2 : 0.0;
        if (K == 1) {
            c0 = q.q[0][0] * w0 + q.q[0][1] * rn1;
        } else {
            c0 = q.q[0][0] * w0 + q.q[0][1] * w1 + q.q[0][2] * rn2 + q.q[0][3] * rn1;
            c1 = q.q[1][0] * w0 + q.q[1][1] * w1 + q.q[1][2] * rn2 + q.q[1][3] * rn1;
        }
        for (int t = 0; t < C; ++t) v[t] += arr(qz, full, t) * c0 + (K == 2 ? arr(qz + 1, full, t) * c1 : 0.0);
    }
    for (int t = 0; t < nr; ++t) x[tr0 + t] = v[t];
    // solve the full chunks
    for (int j = 0; j < full; ++j) {
        std::vector<double> w(f + j * C, f + (j + 1) * C);
        double y1 = H1[j], y2 = H2[j];
        for (int t = 0; t < C; ++t) {
            double y = arr(qs, j, t) * w[t];
            if (K == 2) y += arr(ql + 1, j, t) * y2;
            y += arr(ql, j, t) * y1;
            w[t] = y; y2 = y1; y1 = y;
        }
        double g1 = F1[j], g2 = F2[j];
        for (int t = C - 1; t >= 0; --t) {
            double xx = w[t];
            if (K == 2) xx += arr(qu + 1, j, t) * g2;
            xx += arr(qu, j, t) * g1;
            g2 = g1; g1 = xx;
            if (F.cyclic) xx += arr(qz, j, t) * c0 + (K == 2 ? arr(qz + 1, j, t) * c1 : 0.0);
            w[t] = xx;
        }
        for (int t = 0; t < C; ++t) x[j * C + t] = w[t];
    }
    return 0;
}
