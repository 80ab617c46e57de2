// Device-side parameter structs shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace semcond {

// 1D tables of one scalar type, on the device (see tables.h):
//   lam, a, b: n_I; S, St (= S^T), Sinv, SinvT: n_I x n_I row-major;
//   w: p+1 GLL weights.
// The scalars M_00, K_00, K_0p are passed by value.
template <typename T>
struct DevTab {
    const T* lam;
    const T* a;
    const T* b;
    const T* S;
    const T* St;
    const T* Sinv;
    const T* SinvT;
    const T* w;
    T m0, K00, K0p;
};

// Mesh metric data.  d_e = (h1 h2 h3/8)(lambda, 4/h1^2, 4/h2^2, 4/h3^2)
// (Sec. 3, eq. metriccoeffelement) from per-axis widths and lambda, unless a
// per-element table dcoef[n_e][4] is given.  ax holds per axis and element
// (h/2, 4/h^2), formed on the host, so kernels only multiply.
struct Geo {
    Layout L;
    const double* hx;
    const double* hy;
    const double* hz;
    const double* ax;     // [n1 + n2 + n3][2]
    double lam;
    const double* lam_e;  // nullable, n_e
    const double* dcoef;  // nullable, n_e x 4 (column 0 unused when lam_e is given)
};

// e = e1 + n1 (e2 + n2 e3); element counts stay below 2^31.
__device__ inline void elem_index(const Layout& L, int64_t e, int* e1, int* e2, int* e3) {
    const uint32_t ee = (uint32_t)e, n1 = (uint32_t)L.n1, n2 = (uint32_t)L.n2;
    const uint32_t q = ee / n1, z = q / n2;
    *e1 = (int)(ee - q * n1);
    *e2 = (int)(q - z * n2);
    *e3 = (int)z;
}

// J_e = h1 h2 h3 / 8 (factor of the GLL-lumped element mass matrix).
__device__ inline double elem_jacobian(const Geo& g, int e1, int e2, int e3) {
    const double* a1 = g.ax + 2 * e1;
    const double* a2 = g.ax + 2 * (g.L.n1 + e2);
    const double* a3 = g.ax + 2 * (g.L.n1 + g.L.n2 + e3);
    return a1[0] * a2[0] * a3[0];
}

__device__ inline void elem_metric(const Geo& g, int64_t e, int e1, int e2, int e3, double d[4]) {
    if (g.dcoef) {
        // metric terms from the table; d_0 = J_e lambda_e when lambda_e is also given
        d[0] = g.lam_e ? elem_jacobian(g, e1, e2, e3) * g.lam_e[e] : g.dcoef[4 * e + 0];
        d[1] = g.dcoef[4 * e + 1];
        d[2] = g.dcoef[4 * e + 2];
        d[3] = g.dcoef[4 * e + 3];
        return;
    }
    const double* a1 = g.ax + 2 * e1;
    const double* a2 = g.ax + 2 * (g.L.n1 + e2);
    const double* a3 = g.ax + 2 * (g.L.n1 + g.L.n2 + e3);
    const double J = a1[0] * a2[0] * a3[0];
    d[0] = J * (g.lam_e ? g.lam_e[e] : g.lam);
    d[1] = J * a1[1];
    d[2] = J * a2[1];
    d[3] = J * a3[1];
}

// 1/x from the hardware reciprocal refined by Newton steps (two in FP64, one
// in FP32): relative error within a few units in the last place.
template <typename T>
__device__ inline T recip(T x);
template <>
__device__ inline double recip<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
template <>
__device__ inline float recip<float>(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// a*b + c with one rounding (the CG direction is formed with it wherever it is
// needed, so every copy of it is bitwise the same).
__device__ inline double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ inline void atomic_add(T* p, T v) {
    unsafeAtomicAdd(p, v);
}

// x plus the value of the lane that the data-parallel-primitive control CTRL
// selects (a permutation inside each row of 16 lanes; every lane of the row
// must be active).  Controls used: 0xB1 quad_perm(1,0,3,2) = lane ^ 1,
// 0x4E quad_perm(2,3,0,1) = lane ^ 2, 0x141 row_half_mirror (7 - lane within
// 8), 0x140 row_mirror (15 - lane within 16).  Applied in that order, the first
// 1, 2, 3 or 4 of them leave every lane of an aligned group of 2, 4, 8 or 16
// lanes holding the sum over its group, the same in every lane.
template <int CTRL>
__device__ inline float dpp_add(float x) {
    const int y = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false);
    return x + __builtin_bit_cast(float, y);
}
template <int CTRL>
__device__ inline double dpp_add(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return x + __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16), same in every lane of
// the group.
template <int G, typename T>
__device__ inline T group_sum(T x) {
    if constexpr (G >= 2) x = dpp_add<0xB1>(x);
    if constexpr (G >= 4) x = dpp_add<0x4E>(x);
    if constexpr (G >= 8) x = dpp_add<0x141>(x);
    if constexpr (G >= 16) x = dpp_add<0x140>(x);
    return x;
}

// x plus the value that a row broadcast (CTRL 0x142: lane 15 of the row
// before, 0x143: lane 31) moves into the rows of ROWS; other rows add 0.
template <int CTRL, int ROWS>
__device__ inline float dpp_row_add(float x) {
    const int y = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWS, 0xF, false);
    return x + __builtin_bit_cast(float, y);
}
template <int CTRL, int ROWS>
__device__ inline double dpp_row_add(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
    return x + __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline float lane63(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}
__device__ inline double lane63(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Wave64 sum in a fixed order, returned to every lane: each row of 16 lanes by
// its in-row tree, then rows 1 and 3 add rows 0 and 2, rows 2 and 3 add row 1;
// lane 63 then holds the total.  Every lane of the wave must be active.
template <typename T>
__device__ inline T wave_sum(T v) {
    v = group_sum<16>(v);
    v = dpp_row_add<0x142, 0xA>(v);
    v = dpp_row_add<0x143, 0xC>(v);
    return lane63(v);
}

}  // namespace semcond
