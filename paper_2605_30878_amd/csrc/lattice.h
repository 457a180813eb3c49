// lattice.h -- lattice descriptors of the HIP library (device and host).
//
// D2Q9 velocities and weights as printed in the paper's Appendix A (the
// matrix c and w_i after Eq. A4).  D3Q19 (the paper's three-dimensional
// extension, Section 4): rest (w = 1/3), 6 faces (1/18), 12 edges (1/36),
// cs^2 = 1/3.  The D3Q19 order puts the nine c_z = 0 directions first, in
// the D2Q9 order, then the c_z = +1 and c_z = -1 groups.
#pragma once

#include <cstdint>

namespace lbm {

struct LatD2Q9 {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int NC = 4;  // interpolation corners of a probe point
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

struct LatD3Q19 {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int NC = 8;
    static constexpr int c[19][3] = {
        {0, 0, 0},   {1, 0, 0},  {0, 1, 0},  {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},  {-1, 1, 0},
        {-1, -1, 0}, {1, -1, 0}, {0, 0, 1},  {1, 0, 1},  {0, 1, 1},  {-1, 0, 1}, {0, -1, 1},
        {0, 0, -1},  {1, 0, -1}, {0, 1, -1}, {-1, 0, -1}, {0, -1, -1}};
    static constexpr int opp[19] = {0, 3, 4, 1, 2, 7, 8, 5, 6, 14, 17, 18, 15, 16, 9, 12, 13, 10, 11};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    // The k-th direction (ascending) whose component A equals S.
    template <int A, int S>
    static constexpr int dir_with(int k) {
        for (int i = 0; i < Q; i++)
            if (c[i][A] == S && k-- == 0) return i;
        return -1;
    }
};

// Node classes stored in the flag array.
enum : uint8_t { FLAG_SOLID = 1, FLAG_NEAR_SOLID = 2, FLAG_GHOST = 4 };

}  // namespace lbm
