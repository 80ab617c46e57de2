// Element-cube pieces of the right-hand-side condensation and the interior
// recovery for n_I <= 15 (Algorithm 4): the element cube and the 1D tables in
// LDS, and the line transforms along one axis, as scalar loops or as FP64
// matrix-core products.

#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace semcond {

// The element cube and the 1D tables live in LDS (the tables read at
// wave-uniform indices, as broadcasts); D^-1 is applied once per interior
// node so that the face sums are plain products.  kRhsThreads threads per
// workgroup.

constexpr int kRhsThreads = 256;

template <int NI>
struct RhsSmem {
    static constexpr int n = NI + 2;
    double C[n * n * n];  // C(kk, jj, ii) at (kk n + jj) n + ii
    double A[NI * NI];    // S^T (condensation) or S (recovery), row-major
    double w[n];
    double a[NI], b[NI], lam[NI];
};

template <int NI>
__device__ void rhs_tables(RhsSmem<NI>& sm, const DevTab<double>& tab, const double* __restrict__ A) {
    for (int t = threadIdx.x; t < NI * NI; t += blockDim.x) sm.A[t] = A[t];
    if (threadIdx.x < NI + 2) sm.w[threadIdx.x] = tab.w[threadIdx.x];
    if (threadIdx.x < NI) {
        sm.a[threadIdx.x] = tab.a[threadIdx.x];
        sm.b[threadIdx.x] = tab.b[threadIdx.x];
        sm.lam[threadIdx.x] = tab.lam[threadIdx.x];
    }
}

// x <- A x on the interior part (entries 1 .. n_I) of every line along AXIS
// (0: ii, 1: jj, 2: kk) whose two fixed indices lie in [lo, n - lo).
template <int NI, int AXIS>
__device__ void rhs_lines(double* C, const double* A, int lo) {
    constexpr int n = NI + 2;
    constexpr int st = AXIS == 0 ? 1 : (AXIS == 1 ? n : n * n);
    const int m = n - 2 * lo;
    for (int l = threadIdx.x; l < m * m; l += blockDim.x) {
        const int u = l / m + lo, v = l - (l / m) * m + lo;  // (slow, fast) fixed indices
        const int base = AXIS == 0 ? (u * n + v) * n : (AXIS == 1 ? u * n * n + v : u * n + v);
        double x[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) x[i] = C[base + (1 + i) * st];
#pragma unroll
        for (int o = 0; o < NI; ++o) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NI; ++i) acc += A[o * NI + i] * x[i];
            C[base + (1 + o) * st] = acc;
        }
    }
}

// ---- The same line transforms on the FP64 matrix cores (n_I >= 8) ---------
// For one axis the n_I x n_I matrix M acts on the interior part of every line:
// with the lines as rows, Y = X M^T is a (lines x n_I) by (n_I x n_I) product,
// done in 16 x 16 x 4 FP64 MFMA steps: 16 lines per tile (M dimension), the
// interior index in chunks of 4 (K), the output index (N, n_I <= 15 < 16).
// Operand layout of v_mfma_f64_16x16x4f64 for lane l: A[l % 16][l / 16],
// B[l / 16][l % 16]; result v of the double4 is D[l / 16 + 4 v][l % 16]
// (checked on gfx950 with distinct row and column codes).
// The waves of the workgroup take the tiles in turn; a tile reads and writes
// only its own lines, so one barrier after the pass suffices.

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int NI>
constexpr bool rhs_mfma() { return NI >= 8; }

// B operand of the line transform by M (row-major n_I x n_I): lane l holds
// M[o][i], o = l % 16, i = 4 c + l / 16, for chunk c (0 outside the matrix).
template <int NI>
struct LineMat {
    double b[(NI + 3) / 4];
};

template <int NI>
__device__ inline void line_mat(LineMat<NI>& B, const double* __restrict__ M) {
    const int lane = threadIdx.x & 63, o = lane & 15, i0 = lane >> 4;
#pragma unroll
    for (int c = 0; c < (NI + 3) / 4; ++c) {
        const int i = 4 * c + i0;
        B.b[c] = (o < NI && i < NI) ? M[o * NI + i] : 0.0;
    }
}

template <int n, int AXIS>
__device__ inline int line_base(int u, int v) {
    return AXIS == 0 ? (u * n + v) * n : (AXIS == 1 ? u * n * n + v : u * n + v);
}

// x <- M x on the interior entries (1 .. n_I) of every line along AXIS whose
// two fixed indices lie in [lo, n - lo).
template <int NI, int AXIS>
__device__ void rhs_lines_mfma(double* C, const LineMat<NI>& B, int lo) {
    constexpr int n = NI + 2;
    constexpr int st = AXIS == 0 ? 1 : (AXIS == 1 ? n : n * n);
    constexpr int NC = (NI + 3) / 4;
    const int m = n - 2 * lo, nl = m * m, ntile = (nl + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    for (int tile = wave; tile < ntile; tile += nw) {
        const int La = tile * 16 + row;
        const bool va = La < nl;
        const int ba = va ? line_base<n, AXIS>(La / m + lo, La % m + lo) : 0;
        mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int i = 4 * c + kq;
            const double a = (va && i < NI) ? C[ba + (1 + i) * st] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B.b[c], acc, 0, 0, 0);
        }
        // lane: output index o = row of lines tile*16 + kq + 4 v
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int L = tile * 16 + kq + 4 * v;
            if (L < nl && row < NI) C[line_base<n, AXIS>(L / m + lo, L % m + lo) + (1 + row) * st] = acc[v];
        }
    }
}

// Condensed right-hand-side row of element slot s (faces [6][n_I^2], edges
// [12][n_I], vertices [8], the apply's element numbering) from the
// transformed cube whose interior holds D^-1 F~_I: a face value minus the
// face's line sum through the interior (Table 2), an edge or vertex value as
// it is.  ent / loc: the slot's element entity and its node in the entity.
template <int NI>
__device__ inline double condensed_row(const RhsSmem<NI>& sm, int s, const double* d, int* ent, int* loc) {
    constexpr int n = NI + 2, p = NI + 1, NI2 = NI * NI;
#define C(kk, jj, ii) sm.C[((kk) * n + (jj)) * n + (ii)]
    double val;
    if (s < 6 * NI2) {
        const int fc = s / NI2;
        *loc = s - fc * NI2;
        *ent = fc;
        const int s1 = *loc / NI, s2 = *loc - (*loc / NI) * NI;
        const double* c = (fc & 1) ? sm.b : sm.a;
        const int side = (fc & 1) ? p : 0;
        double acc = 0.0;
        if (fc < 2) {  // (k, j), sum over i
#pragma unroll
            for (int m = 0; m < NI; ++m) acc += c[m] * C(1 + s1, 1 + s2, 1 + m);
            val = C(1 + s1, 1 + s2, side) - d[1] * acc;
        } else if (fc < 4) {  // (k, i), sum over j
#pragma unroll
            for (int m = 0; m < NI; ++m) acc += c[m] * C(1 + s1, 1 + m, 1 + s2);
            val = C(1 + s1, side, 1 + s2) - d[2] * acc;
        } else {  // (j, i), sum over k
#pragma unroll
            for (int m = 0; m < NI; ++m) acc += c[m] * C(1 + m, 1 + s1, 1 + s2);
            val = C(side, 1 + s1, 1 + s2) - d[3] * acc;
        }
    } else if (s < 6 * NI2 + 12 * NI) {
        const int q = (s - 6 * NI2) / NI;
        *loc = s - 6 * NI2 - q * NI;
        *ent = 6 + q;
        if (q < 4) {
            const int jb = q & 1, kb = q >> 1;
            val = C(kb * p, jb * p, 1 + *loc);
        } else if (q < 8) {
            const int ib = (q - 4) & 1, kb = (q - 4) >> 1;
            val = C(kb * p, 1 + *loc, ib * p);
        } else {
            const int ib = (q - 8) & 1, jb = (q - 8) >> 1;
            val = C(1 + *loc, jb * p, ib * p);
        }
    } else {
        const int q = s - 6 * NI2 - 12 * NI;
        *ent = 18 + q;
        *loc = 0;
        val = C((q >> 2) * p, ((q >> 1) & 1) * p, (q & 1) * p);
    }
#undef C
    return val;
}

}  // namespace semcond
