// d3q19.hpp -- D3Q19 velocity set of the library (device and host).
//
// The paper works with the D3Q19 stencil (Sec. 1; Table 8) without printing
// its velocities; this is the standard set.  The order is the library's
// convention, fixed in lbm355.h: rest, then each moving direction followed
// by its opposite.
#pragma once

#include <cstdint>

namespace lbm {

constexpr int Q = 19;

__host__ __device__ constexpr int cx(int i)
{
    constexpr int t[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int cy(int i)
{
    constexpr int t[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
__host__ __device__ constexpr int cz(int i)
{
    constexpr int t[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
// opposite direction: pairs (1,2), (3,4), ... (17,18)
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// weights 1/3, 1/18, 1/36 (exact doubles of these fractions)
__host__ __device__ constexpr double wd(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Offset o_i = max(-c_i, 0) (componentwise) of the esoteric twist: f_i of
// node x is stored at cell x + o_i.  o_{opp i} - o_i = c_i.
__host__ __device__ constexpr int ox(int i) { return cx(i) < 0 ? 1 : 0; }
__host__ __device__ constexpr int oy(int i) { return cy(i) < 0 ? 1 : 0; }
__host__ __device__ constexpr int oz(int i) { return cz(i) < 0 ? 1 : 0; }

// The seven cells an esoteric-twist update touches, x + {0, ex, ey, ez,
// ex+ey, ex+ez, ey+ez}; et_cell(ox, oy, oz) gives the slot number 0..6.
__host__ __device__ constexpr int et_cell(int a, int b, int c)
{
    return (a + b + c == 0) ? 0
         : (a + b + c == 1) ? (a ? 1 : (b ? 2 : 3))
         : (!c ? 4 : (!b ? 5 : 6));
}

} // namespace lbm
