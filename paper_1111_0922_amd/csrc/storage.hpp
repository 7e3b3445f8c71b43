// storage.hpp -- PDF storage precisions and memory layouts.
//
// Precisions: FP64 (compute FP64), FP32 (compute FP32), and the shifted
// deviations h_i = (f_i - w_i) * sigma stored in binary16 (FP16S) or binary32
// (F32S), both computed in FP32.
// Layouts (Sec. 1): SoA keeps one array per direction, element j * pitch + a;
// AoS keeps the 19 values of a cell together, element a * 19 + j.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "d3q19.hpp"

namespace lbm {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_F16S = 2, P_F32S = 3 };
// L_BLK: the blocked SoA order of indirect lattices (slot_index in kernels.hpp);
// the public layouts are SoA and AoS, and an indirect SoA grid is stored as
// L_SOA or L_BLK
enum Lay : int { L_SOA = 0, L_AOS = 1, L_BLK = 2 };

template <int P>
struct Store;

// rt: the register a raw stored value is held in between its load and its
// conversion.  binary16 values stay in a full 32-bit register (zero-extended
// 16-bit load): packing two of them per register would chain the loads.
template <>
struct Store<P_F64> {
    using st = double;
    using ct = double;
    using rt = double;
    __device__ static rt raw(st x) { return x; }
    __device__ static st unraw(rt r) { return r; }
    __device__ static ct load_raw(rt r) { return r; }
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
    using rt = float;
    __device__ static rt raw(st x) { return x; }
    __device__ static st unraw(rt r) { return r; }
    __device__ static ct load_raw(rt r) { return r; }
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
    using rt = uint32_t;
    __device__ static rt raw(st x) { return (uint32_t)__builtin_bit_cast(uint16_t, x); }
    __device__ static st unraw(rt r) { return __builtin_bit_cast(_Float16, (uint16_t)r); }
    __device__ static ct load_raw(rt r) { return (float)unraw(r); }
    static constexpr bool shifted = true;
    __device__ static ct load(st x) { return (float)x; }
    __device__ static st save(ct v) { return (_Float16)v; }
    // f = w_i + h / sigma
    __device__ static double to_canon(st x, int i, double sigma) { return wd(i) + (double)x / sigma; }
    // h = (f - w_i) * sigma, rounded once from FP64 to binary16
    __device__ static st from_canon(double f, int i, double sigma) { return (_Float16)((f - wd(i)) * sigma); }
};

// PDF traffic of the direct SoA update kernels, and of node-local kernels on
// indirect SoA grids, streams through the caches exactly once per step
// (every line is read and written whole), so their loads and stores carry
// the nontemporal hint.  Indirect gathers and AoS records reuse partly used
// lines across neighbouring nodes; there the hint costs traffic and is not
// used.  LBM_NT_LOAD / LBM_NT_STORE = 0 at build
// time disable it everywhere (measurements of build variants).
#ifndef LBM_NT_LOAD
#define LBM_NT_LOAD 1
#endif
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif

template <bool NT, typename T>
__device__ __forceinline__ T pdf_load(const T *p)
{
    if constexpr (NT && LBM_NT_LOAD)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void pdf_store(T *p, T v)
{
    if constexpr (NT && LBM_NT_STORE)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// load of one stored PDF into its raw register
template <bool NT, class S>
__device__ __forceinline__ typename S::rt pdf_load_raw(const typename S::st *p)
{
    if constexpr (sizeof(typename S::st) == 2) {
        const uint16_t *q = reinterpret_cast<const uint16_t *>(p);
        return (uint32_t)pdf_load<NT>(q);
    } else {
        return pdf_load<NT>(p);
    }
}

template <>
struct Store<P_F32S> {
    using st = float;
    using ct = float;
    using rt = float;
    static constexpr bool shifted = true;
    __device__ static rt raw(st x) { return x; }
    __device__ static st unraw(rt r) { return r; }
    __device__ static ct load_raw(rt r) { return r; }
    __device__ static ct load(st x) { return x; }
    __device__ static st save(ct v) { return v; }
    __device__ static double to_canon(st x, int i, double sigma) { return wd(i) + (double)x / sigma; }
    __device__ static st from_canon(double f, int i, double sigma) { return (float)((f - wd(i)) * sigma); }
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
