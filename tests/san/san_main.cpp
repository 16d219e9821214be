// san_main.cpp -- the host side of libbandbatch (factorisation, tables,
// argument checks, decomposition plans, error reporting), the CPU replay of
// the GPU decompositions (tests/emu/chunk_emu.cpp) and the FP64 oracle, run
// together in one program built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  No device is used:
// every library call made here returns before its first HIP call.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../../include/bandbatch.h"

extern "C" int emu_solve(int kind, const double *a, const double *b, const double *c,
                         const double *d, const double *e, int64_t n, int adjoint, int C,
                         const double *f, double *x);
extern "C" int emu_solve_long(int kind, const double *a, const double *b, const double *c,
                              const double *d, const double *e, int64_t n, int adjoint, int C,
                              const double *f, double *x);
extern "C" int oracle_solve_batch(int kind, int64_t n, int64_t m, int64_t ld, const double *a,
                                  const double *b, const double *c, const double *d,
                                  const double *e, const double *rhs, double *x);
extern "C" int oracle_ch_step_batch(int64_t n, int64_t m, int64_t ld, double sigma, double alpha,
                                    const double *c_in, double *c_out);

static int failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

struct Bands {
    std::vector<double> v[5];
};

static Bands dominant(int K, int64_t n, std::mt19937_64 &g)
{
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    Bands b;
    const int nb = 2 * K + 1;
    for (int q = 0; q < nb; ++q) b.v[q].resize(n);
    for (int64_t i = 0; i < n; ++i) {
        double off = 0.0;
        for (int q = 0; q < nb; ++q)
            if (q != K) {
                b.v[q][i] = u(g);
                off += std::fabs(b.v[q][i]);
            }
        b.v[K][i] = (off + 1.0) * (u(g) < 0 ? -1.0 : 1.0);
    }
    for (int q = nb; q < 5; ++q) b.v[q].assign(n, 0.0);
    return b;
}

static bb_status make(int kind, const Bands &b, int64_t n, bb_factor *f)
{
    switch (kind) {
    case 0: return bb_factor_shared_tri(b.v[0].data(), b.v[1].data(), b.v[2].data(), n, f);
    case 1: return bb_factor_shared_tri_cyclic(b.v[0].data(), b.v[1].data(), b.v[2].data(), n, f);
    case 2:
        return bb_factor_shared_penta(b.v[0].data(), b.v[1].data(), b.v[2].data(), b.v[3].data(),
                                      b.v[4].data(), n, f);
    default:
        return bb_factor_shared_penta_cyclic(b.v[0].data(), b.v[1].data(), b.v[2].data(),
                                             b.v[3].data(), b.v[4].data(), n, f);
    }
}

static double rel(const std::vector<double> &x, const std::vector<double> &r)
{
    double num = 0, den = 0;
    for (size_t i = 0; i < x.size(); ++i) {
        num += (x[i] - r[i]) * (x[i] - r[i]);
        den += r[i] * r[i];
    }
    return std::sqrt(num / (den > 0 ? den : 1.0));
}

int main()
{
    std::mt19937_64 g(2107053950);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    const int64_t sizes[] = {1, 2, 3, 4, 5, 7, 33, 64, 65, 257, 1000, 1024, 1025, 2048, 2049, 5000};
    // never dereferenced: every call below fails its argument checks first
    // or has m = 0
    void *fake = (void *)0x1000, *other = (void *)0x2000;
    double *dfake = (double *)fake, *dother = (double *)other;
    double *dfar = (double *)(uintptr_t(1) << 44);   // beyond every range the checks form
    // factors of every kind and size, their plans and info, argument errors
    for (int kind = 0; kind < 4; ++kind) {
        const int K = kind < 2 ? 1 : 2;
        for (int64_t n : sizes) {
            Bands b = dominant(K, n, g);
            bb_factor f = nullptr;
            const bb_status st = make(kind, b, n, &f);
            const int64_t nmin = kind == 1 ? 3 : kind == 3 ? 5 : 1;
            if (n < nmin) {
                CHECK(st == BB_ERR_ARG && f == nullptr);
                continue;
            }
            CHECK(st == BB_OK && f != nullptr);
            int64_t nn = 0;
            int32_t kk = -1, chunk = 0, lanes = 0, waves = 0, scalar = 0;
            CHECK(bb_factor_info(f, &nn, &kk, &chunk) == BB_OK && nn == n && kk == kind);
            for (int64_t m : {int64_t(1), int64_t(100), int64_t(1) << 16})
                for (int what = 0; what < 2; ++what)
                    for (int p = 0; p < 4; ++p) {
                        CHECK(bb_plan(f, m, what, (bb_precision)p, &chunk, &lanes, &waves,
                                      &scalar) == BB_OK);
                        CHECK(chunk >= 4 && (int64_t)chunk * lanes >= n && waves >= 1);
                    }
            CHECK(bb_plan(f, 0, 0, BB_F64, nullptr, nullptr, nullptr, nullptr) == BB_ERR_ARG);
            CHECK(bb_plan(f, 5, 2, BB_F64, nullptr, nullptr, nullptr, nullptr) == BB_ERR_ARG);
            auto solve = K == 1 ? bb_solve_batch_tri : bb_solve_batch_penta;
            CHECK(solve(f, nullptr, nullptr, 0, 1, BB_F64, nullptr) == BB_OK);      // m = 0
            CHECK(solve(f, fake, other, 8, 4, BB_F64, nullptr) == BB_ERR_ARG);     // ld < m
            CHECK(solve(f, nullptr, other, 4, 4, BB_F64, nullptr) == BB_ERR_ARG);
            CHECK(solve(f, fake, other, 4, 4, (bb_precision)9, nullptr) == BB_ERR_ARG);
            CHECK(solve(f, fake, fake, 4, 4, BB_F32_RHS_REFINE, nullptr) == BB_ERR_ARG);
            auto wrong = K == 1 ? bb_solve_batch_penta : bb_solve_batch_tri;
            CHECK(wrong(f, fake, other, 4, 4, BB_F64, nullptr) == BB_ERR_ARG);
            CHECK(bb_band_grad(f, dfake, dfake, 4, 4, nullptr, nullptr, 0, nullptr) == BB_ERR_ARG);
            for (int64_t m : {int64_t(1), int64_t(100), int64_t(5000), int64_t(1) << 16}) {
                const size_t ws = bb_adjoint_band_grad_workspace_bytes(f, m, m);
                CHECK(ws >= (size_t)(2 * K + 1) * n * sizeof(double));
                CHECK(bb_adjoint_band_grad_fused(f, m) == 0 || bb_adjoint_band_grad_fused(f, m) == 1);
                CHECK(bb_adjoint_band_grad(f, dfake, dother, dfar, m, m, 2, dother, fake, ws - 1,
                                           nullptr) == BB_ERR_ARG);       // workspace too small
                CHECK(bb_adjoint_band_grad(f, dfake, dother, dother, m, m, 2, dother, fake, ws,
                                           nullptr) == BB_ERR_ARG);       // lam overlaps traj
            }
            CHECK(bb_adjoint_band_grad(f, dfake, dother, dfar, 4, 4, 0, dother, fake, 1 << 30,
                                       nullptr) == BB_ERR_ARG);           // steps < 1
            CHECK(bb_adjoint_band_grad(f, nullptr, nullptr, nullptr, 0, 1, 1, dother, nullptr, 0,
                                       nullptr) == BB_OK);                // m = 0
            const bool long_sys = n > (K == 1 ? 2048 : 1024);
            if (long_sys) {
                CHECK(solve(f, fake, other, 4, 4, BB_F32_REFINE, nullptr) == BB_ERR_UNSUPPORTED);
                CHECK(solve(f, fake, fake, 4, 4, BB_F64, nullptr) == BB_ERR_UNSUPPORTED);
            }
            const double w[5] = {0.1, 0.2, 0.4, 0.2, 0.1};
            CHECK(bb_cn_step(f, w, dfake, dother, 8, 4, 1, nullptr) == BB_ERR_ARG);
            CHECK(bb_cn_step(f, nullptr, dfake, dother, 4, 4, 1, nullptr) == BB_ERR_ARG);
            CHECK(bb_factor_destroy(f) == BB_OK);
        }
    }
    // zero pivots and singular periodic capacitances
    {
        std::vector<double> a(8, 1.0), b(8, 0.0), c(8, 1.0);
        bb_factor f = nullptr;
        CHECK(bb_factor_shared_tri(a.data(), b.data(), c.data(), 8, &f) == BB_ERR_ZERO_PIVOT);
        CHECK(std::string(bb_last_error_message()).find("pivot") != std::string::npos);
        b.assign(8, -2.0);   // periodic second difference: singular
        CHECK(bb_factor_shared_tri_cyclic(a.data(), b.data(), c.data(), 8, &f) != BB_OK);
        CHECK(f == nullptr);
        std::vector<double> e(8, 1.0), d(8, -4.0), cc(8, 6.0);   // periodic fourth difference
        CHECK(bb_factor_shared_penta_cyclic(e.data(), d.data(), cc.data(), d.data(), e.data(), 8,
                                            &f) != BB_OK);
        CHECK(bb_factor_shared_tri(nullptr, b.data(), c.data(), 8, &f) == BB_ERR_ARG);
        CHECK(bb_factor_shared_tri(a.data(), b.data(), c.data(), bb_max_n() + 1, &f) ==
              BB_ERR_UNSUPPORTED);
        for (int s = -7; s <= 1; ++s) CHECK(bb_status_string((bb_status)s) != nullptr);
    }
    // the Cahn-Hilliard factor, short and long
    for (int64_t n : {int64_t(5), int64_t(256), int64_t(1024), int64_t(1025), int64_t(4096)}) {
        bb_factor f = nullptr;
        double sigma = 0, alpha = 0;
        CHECK(bb_factor_ch(n, 2 * M_PI, 0.01, 1e-3, &f, &sigma, &alpha) == BB_OK);
        const double dx = 2 * M_PI / n;
        CHECK(std::fabs(alpha - 1e-3 / (dx * dx)) <= 1e-12 * alpha);
        CHECK(bb_ch_step(f, dfake, dother, 4, 4, alpha, 0, nullptr) == BB_ERR_ARG);
        CHECK(bb_ch_step(f, nullptr, nullptr, 0, 1, alpha, 1, nullptr) == BB_OK);
        if (n > 1024) CHECK(bb_ch_step(f, dfake, dother, 4, 4, alpha, 2, nullptr) == BB_ERR_UNSUPPORTED);
        CHECK(bb_factor_destroy(f) == BB_OK);
    }
    CHECK(bb_factor_ch(4, 1.0, 0.01, 1e-3, nullptr, nullptr, nullptr) == BB_ERR_ARG);
    // the decompositions replayed on the host against the oracle
    for (int kind = 0; kind < 4; ++kind) {
        const int K = kind < 2 ? 1 : 2;
        for (int64_t n : {int64_t(7), int64_t(100), int64_t(257), int64_t(1000), int64_t(3001)}) {
            Bands b = dominant(K, n, g);
            std::vector<double> f(n), x(n), r(n);
            for (auto &v : f) v = u(g);
            CHECK(oracle_solve_batch(kind, n, 1, 1, b.v[0].data(), b.v[1].data(), b.v[2].data(),
                                     b.v[3].data(), b.v[4].data(), f.data(), r.data()) == 0);
            for (int C : {4, 16, 64}) {
                if ((n + C - 1) / C <= 64) {
                    CHECK(emu_solve(kind, b.v[0].data(), b.v[1].data(), b.v[2].data(),
                                    b.v[3].data(), b.v[4].data(), n, 0, C, f.data(),
                                    x.data()) == 0);
                    CHECK(rel(x, r) < 1e-13);
                }
                if (C >= 16 && (n + C - 1) / C >= 2) {
                    CHECK(emu_solve_long(kind, b.v[0].data(), b.v[1].data(), b.v[2].data(),
                                         b.v[3].data(), b.v[4].data(), n, 0, C, f.data(),
                                         x.data()) == 0);
                    CHECK(rel(x, r) < 1e-13);
                }
            }
        }
    }
    {
        const int64_t n = 256, m = 3;
        std::vector<double> c(n * m), o(n * m);
        for (auto &v : c) v = 0.1 * u(g);
        CHECK(oracle_ch_step_batch(n, m, m, 27.5575, 1.66005, c.data(), o.data()) == 0);
    }
    std::printf("%s: %d failed checks\n", failures ? "sanitizer run FAILED" : "sanitizer run ok",
                failures);
    return failures ? 1 : 0;
}
