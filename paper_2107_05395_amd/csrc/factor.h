// factor.h -- host-side shared-matrix factor of libbandbatch.
//
// The matrix is factorised once, on the host, in double (Section 3.1
// pre-factorisation; Section 4.1 LR factorisation; Appendix A/B), and turned
// into the per-row recurrence coefficients of internal.h for both the solve
// and the transposed (adjoint) solve.  Periodic matrices are split as
// A = A' + U V^T (Section 3.3; rank-2 analogue for the Section 5.1 matrix) and
// the correction vectors and capacitance inverse are precomputed here too.
#pragma once

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace bb {

enum Kind : int { kTri = 0, kTriCyclic = 1, kPenta = 2, kPentaCyclic = 3 };

// Recurrence rows of one direction (internal.h): forward s, l1, l2; backward u1, u2.
struct Recurrence {
    std::vector<double> s, l1, l2, u1, u2;
};

// Periodic correction of one direction: x = y - Z s, s = Q (ends of y).
struct Correction {
    std::vector<double> z0, z1;
    CyclicQ q{};
};

struct Direction {
    Recurrence rec;
    Correction cor;
};

enum Status : int { kOk = 0, kErrArg = -1, kErrPivot = -2, kErrCapacitance = -3 };

struct DeviceTable {
    void *ptr = nullptr;
    int64_t elems = 0;
};

struct Factor {
    int kind = kTri;
    int K = 1;
    bool cyclic = false;
    int64_t n = 0;
    std::vector<double> band[5];   // original matrix, 2K+1 bands, entries outside the matrix zeroed
    Corners corners{};             // original periodic corners (refinement residual)
    Direction primal, adjoint;
    // factor of the shared matrix in the paper's quantities (kept for the
    // thread-per-system baseline kernel): 1/b^, a/b^, c^ (tri only)
    std::vector<double> rhat, aprime, chat;

    std::mutex mu;
    // (device, adjoint?, f32?, C, with residual bands?) -> device table
    std::map<std::tuple<int, int, int, int, int>, DeviceTable> dev;
    std::map<int, DeviceTable> dev_paper;   // per device: rhat | aprime | chat

    ~Factor();
};

// Build a factor; returns kOk or a negative Status with a message in `err`.
int make_factor(int kind, const double *const bands[5], int64_t n, Factor &f, std::string &err);

// Chunk size for a solve of n rows (rows per lane), power of two in
// [kChunkMin, kChunkMax]; lanes per system P = ceil(n / C) rounded up to a
// power of two, at most 64.
int choose_chunk(int64_t n, int cmax);
int lanes_for(int64_t n, int C);

// Host table in the layout of internal.h (T = double or float), optionally
// followed by nothing else; residual bands are built separately.
std::vector<double> build_table(const Direction &d, int K, bool cyclic, int64_t n, int C, int P);
std::vector<double> build_band_table(const Factor &f, int C, int P);

}  // namespace bb
