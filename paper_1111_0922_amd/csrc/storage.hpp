// storage.hpp -- PDF storage precisions and memory layouts.
//
// Precisions: FP64 (compute FP64), FP32 (compute FP32), FP16S: the shifted
// deviation h_i = (f_i - w_i) * sigma in binary16, computed in FP32.
// Layouts (Sec. 1): SoA keeps one array per direction, element j * pitch + a;
// AoS keeps the 19 values of a cell together, element a * 19 + j.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "d3q19.hpp"

namespace lbm {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_F16S = 2 };
enum Lay : int { L_SOA = 0, L_AOS = 1 };

template <int P>
struct Store;

template <>
struct Store<P_F64> {
    using st = double;
    using ct = double;
    static constexpr bool shifted = false;
    __device__ static ct load(st x) { return x; }
    __device__ static st save(ct v) { return v; }
    __device__ static double to_canon(st x, int, double) { return x; }
    __device__ static st from_canon(double f, int, double) { return f; }
};

template <>
struct Store<P_F32> {
    using st = float;
    using ct = float;
    static constexpr bool shifted = false;
    __device__ static ct load(st x) { return x; }
    __device__ static st save(ct v) { return v; }
    __device__ static double to_canon(st x, int, double) { return (double)x; }
    __device__ static st from_canon(double f, int, double) { return (float)f; }
};

template <>
struct Store<P_F16S> {
    using st = _Float16;
    using ct = float;
    static constexpr bool shifted = true;
    __device__ static ct load(st x) { return (float)x; }
    __device__ static st save(ct v) { return (_Float16)v; }
    // f = w_i + h / sigma
    __device__ static double to_canon(st x, int i, double sigma) { return wd(i) + (double)x / sigma; }
    // h = (f - w_i) * sigma, rounded once from FP64 to binary16
    __device__ static st from_canon(double f, int i, double sigma) { return (_Float16)((f - wd(i)) * sigma); }
};

template <int L>
__device__ __forceinline__ int64_t elem(int j, int64_t a, int64_t pitch)
{
    if constexpr (L == L_SOA)
        return (int64_t)j * pitch + a;
    else
        return a * Q + j;
}

} // namespace lbm
