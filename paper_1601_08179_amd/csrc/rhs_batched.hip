// Right-hand-side condensation and interior recovery (Algorithm 4, first and
// second loops) for 8 <= n_I <= 12 with R right-hand sides per workgroup.
//
// A workgroup takes one element and a batch of R right-hand sides.  What does
// not depend on the right-hand side is set up once: the 1D tables and the
// line-transform matrix (with the interior quadrature weights folded in) in
// LDS, its matrix-core operand, the element's entity bases, every thread's node
// offsets, D^-1 at its interior points and its output addresses in registers.
// Per right-hand side the element values go through the LDS cube: the FP64
// matrix-core line transforms along the three axes (rhs_lines.h), D^-1, and
// the face line sums or the back transform; the loads of the next right-hand
// side are issued before the current one is transformed.  R is chosen per
// context and k by timing (api.cpp); every right-hand side's arithmetic is the
// same for any R.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"
#include "layout.h"
#include "rhs_lines.h"

namespace semcond {

// Waves per SIMD asked of the compiler: 3 fits n_I <= 11 without spills
// (165 and 144 VGPRs at n_I = 11); n_I = 12 keeps its own choice.
template <int NI>
constexpr int rhs_mb_waves() { return NI <= 11 ? 3 : 1; }

template <int NI>
__global__ __launch_bounds__(kRhsThreads) __attribute__((amdgpu_waves_per_eu(rhs_mb_waves<NI>())))
void k_condense_rhs_mb(Geo g, DevTab<double> tab,
                                                                 const double* __restrict__ f, int64_t N,
                                                                 double* __restrict__ fhat, int k, int R,
                                                                 double* __restrict__ slots, int64_t qlen,
                                                                 uint32_t ns, int64_t rs) {
    constexpr int n = NI + 2, p = NI + 1, NI2 = NI * NI, NI3 = NI2 * NI, n3 = n * n * n;
    constexpr int nslot = 6 * NI2 + 12 * NI + 8;
    constexpr int T = kRhsThreads;
    constexpr int QC = (n3 + T - 1) / T, QD = (NI3 + T - 1) / T;
    static_assert(QC <= 32, "boundary counts are packed two bits each into 64 bits");
    __shared__ RhsSmem<NI> sm;
    __shared__ int64_t ebase[26];
    __shared__ int econ[26];
    __shared__ double wfac[4];  // J w_0^m for a node with m boundary indices (w_p = w_0)
    const Layout& L = g.L;
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int r0 = (int)blockIdx.y * R, r1 = min(k, r0 + R);
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    const double J = elem_jacobian(g, e1, e2, e3);
    // S^T with the interior weights folded in: A[o][i] = S^T[o][i] w_{1+i}
    for (int t = tid; t < NI2; t += T) sm.A[t] = tab.St[t] * tab.w[1 + t % NI];
    if (tid < NI) {
        sm.a[tid] = tab.a[tid];
        sm.b[tid] = tab.b[tid];
        sm.lam[tid] = tab.lam[tid];
    }
    if (tid < 26) {
        bool c;
        element_entity(L, e1, e2, e3, tid, &ebase[tid], &c);
        econ[tid] = c ? 1 : 0;
    }
    if (tid < 4) {
        double x = J;
        for (int m = 0; m < tid; ++m) x *= tab.w[0];
        wfac[tid] = x;
    }
    __syncthreads();

    // cube nodes of the thread: offsets from the element's first node (the
    // launcher checks N < 2^32) and boundary-index counts
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    const int64_t node0 = (int64_t)e1 * p + N1 * ((int64_t)e2 * p + N2 * ((int64_t)e3 * p));
    uint32_t coff[QC];
    uint64_t bcnt = 0;
#pragma unroll
    for (int q = 0; q < QC; ++q) {
        const int idx = tid + T * q;
        const int ii = idx % n, jj = (idx / n) % n, kk = idx / (n * n);
        coff[q] = idx < n3 ? (uint32_t)(ii + N1 * (jj + N2 * kk)) : 0u;
        const int m = (ii == 0 || ii == p) + (jj == 0 || jj == p) + (kk == 0 || kk == p);
        bcnt |= (uint64_t)m << (2 * q);
    }
    // D^-1 at the thread's interior points
    double dinv[QD];
#pragma unroll
    for (int q = 0; q < QD; ++q) {
        const int idx = tid + T * q < NI3 ? tid + T * q : 0;
        const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
        dinv[q] = recip<double>(d[0] + d[1] * sm.lam[i] + d[2] * sm.lam[j] + d[3] * sm.lam[kk]);
    }
    LineMat<NI> B;
    line_mat<NI>(B, sm.A);

    double pre[QC];
    auto issue = [&](int r) __attribute__((always_inline)) {
        const double* fb = f + (int64_t)r * N + node0;
#pragma unroll
        for (int q = 0; q < QC; ++q) pre[q] = tid + T * q < n3 ? fb[coff[q]] : 0.0;
    };
    if (r0 < r1) issue(r0);
    for (int r = r0; r < r1; ++r) {
#pragma unroll
        for (int q = 0; q < QC; ++q)
            if (tid + T * q < n3) sm.C[tid + T * q] = wfac[(bcnt >> (2 * q)) & 3] * pre[q];
        __syncthreads();
        if (r + 1 < r1) issue(r + 1);
        rhs_lines_mfma<NI, 0>(sm.C, B, 0);
        __syncthreads();
        rhs_lines_mfma<NI, 1>(sm.C, B, 0);
        __syncthreads();
        rhs_lines_mfma<NI, 2>(sm.C, B, 0);
        __syncthreads();
        // interior: V = D^-1 F~_I
#pragma unroll
        for (int q = 0; q < QD; ++q) {
            const int idx = tid + T * q;
            if (idx < NI3) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                sm.C[((1 + kk) * n + 1 + j) * n + 1 + i] *= dinv[q];
            }
        }
        __syncthreads();
        // one element slot after the other (unrolled, the line sums of several
        // slots would hold their LDS values in registers together)
#pragma unroll 1
        for (int s = tid; s < nslot; s += T) {
            int ent, loc;
            const double val = condensed_row<NI>(sm, s, d, &ent, &loc);
            if (econ[ent]) continue;
            const uint32_t node = (uint32_t)(ebase[ent] + loc);
            if (slots)
                slots[(int64_t)r * qlen + slot_addr(L, node, entity_slot(ent))] = val;
            else
                atomic_add(&fhat[(int64_t)node * ns + (int64_t)r * rs], val);
        }
        __syncthreads();  // the next right-hand side rewrites the cube
    }
}

template <int NI>
__global__ __launch_bounds__(kRhsThreads) __attribute__((amdgpu_waves_per_eu(rhs_mb_waves<NI>())))
void k_recover_interior_mb(Geo g, DevTab<double> tab,
                                                                     const double* __restrict__ f, int64_t N,
                                                                     const double* __restrict__ xs,
                                                                     double* __restrict__ u, int k, int R,
                                                                     int keep_con, uint32_t ns, int64_t rs) {
    constexpr int n = NI + 2, p = NI + 1, NI2 = NI * NI, NI3 = NI2 * NI;
    constexpr int T = kRhsThreads;
    constexpr int QI = (NI3 + T - 1) / T, QF = (6 * NI2 + T - 1) / T;
    __shared__ RhsSmem<NI> sm;
    __shared__ double UF[6 * NI2];  // the element's six faces of u~_B
    __shared__ double Sb[NI * NI];  // S (back transform), row-major
    __shared__ int64_t fb[6];
    __shared__ int fcon[6];
    const Layout& L = g.L;
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const int r0 = (int)blockIdx.y * R, r1 = min(k, r0 + R);
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    const double J = elem_jacobian(g, e1, e2, e3);
    for (int t = tid; t < NI2; t += T) {
        sm.A[t] = tab.St[t] * tab.w[1 + t % NI];  // forward: S^T diag(w_interior)
        Sb[t] = tab.S[t];
    }
    if (tid < NI) {
        sm.a[tid] = tab.a[tid];
        sm.b[tid] = tab.b[tid];
        sm.lam[tid] = tab.lam[tid];
    }
    if (tid < 6) {
        bool c;
        element_entity(L, e1, e2, e3, tid, &fb[tid], &c);
        fcon[tid] = c && !keep_con ? 1 : 0;
    }
    __syncthreads();

    // interior nodes of the thread (offsets from the element's first interior
    // node) with D^-1 there, and its face values (skeleton node or ~0: zero)
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    const int64_t node1 = ((int64_t)e1 * p + 1) + N1 * (((int64_t)e2 * p + 1) + N2 * ((int64_t)e3 * p + 1));
    uint32_t ioff[QI];
    double dinv[QI];
#pragma unroll
    for (int q = 0; q < QI; ++q) {
        const int idx = tid + T * q < NI3 ? tid + T * q : 0;
        const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
        ioff[q] = (uint32_t)(i + N1 * (j + N2 * kk));
        dinv[q] = recip<double>(d[0] + d[1] * sm.lam[i] + d[2] * sm.lam[j] + d[3] * sm.lam[kk]);
    }
    uint32_t fnode[QF];
#pragma unroll
    for (int q = 0; q < QF; ++q) {
        const int s = tid + T * q;
        const int fc = s / NI2 < 6 ? s / NI2 : 0;
        fnode[q] = (s < 6 * NI2 && !fcon[fc]) ? (uint32_t)(fb[fc] + (s - fc * NI2)) : ~0u;
    }
    LineMat<NI> Bf, Bb;
    line_mat<NI>(Bf, sm.A);
    line_mat<NI>(Bb, Sb);

    double pf[QI], pu[QF];
    auto issue = [&](int r) __attribute__((always_inline)) {
        const double* fr = f + (int64_t)r * N + node1;
#pragma unroll
        for (int q = 0; q < QI; ++q) pf[q] = tid + T * q < NI3 ? fr[ioff[q]] : 0.0;
#pragma unroll
        for (int q = 0; q < QF; ++q) pu[q] = fnode[q] != ~0u ? xs[(int64_t)fnode[q] * ns + (int64_t)r * rs] : 0.0;
    };
#define C(kk, jj, ii) sm.C[((kk) * n + (jj)) * n + (ii)]
    if (r0 < r1) issue(r0);
    for (int r = r0; r < r1; ++r) {
#pragma unroll
        for (int q = 0; q < QI; ++q) {
            const int idx = tid + T * q;
            if (idx < NI3) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                C(1 + kk, 1 + j, 1 + i) = J * pf[q];
            }
        }
#pragma unroll
        for (int q = 0; q < QF; ++q)
            if (tid + T * q < 6 * NI2) UF[tid + T * q] = pu[q];
        __syncthreads();
        if (r + 1 < r1) issue(r + 1);
        // F~_I: the interior lines only (the boundary entries do not reach the interior)
        rhs_lines_mfma<NI, 0>(sm.C, Bf, 1);
        __syncthreads();
        rhs_lines_mfma<NI, 1>(sm.C, Bf, 1);
        __syncthreads();
        rhs_lines_mfma<NI, 2>(sm.C, Bf, 1);
        __syncthreads();
        // u~_I = D^-1 (F~_I - H~_IB u~_B) (Table 2)
#pragma unroll
        for (int q = 0; q < QI; ++q) {
            const int idx = tid + T * q;
            if (idx < NI3) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                const double uc = d[1] * (sm.a[i] * UF[kk * NI + j] + sm.b[i] * UF[NI2 + kk * NI + j]) +
                                  d[2] * (sm.a[j] * UF[2 * NI2 + kk * NI + i] + sm.b[j] * UF[3 * NI2 + kk * NI + i]) +
                                  d[3] * (sm.a[kk] * UF[4 * NI2 + j * NI + i] + sm.b[kk] * UF[5 * NI2 + j * NI + i]);
                C(1 + kk, 1 + j, 1 + i) = (C(1 + kk, 1 + j, 1 + i) - uc) * dinv[q];
            }
        }
        __syncthreads();
        // u_I = (S (x) S (x) S) u~_I
        rhs_lines_mfma<NI, 0>(sm.C, Bb, 1);
        __syncthreads();
        rhs_lines_mfma<NI, 1>(sm.C, Bb, 1);
        __syncthreads();
        rhs_lines_mfma<NI, 2>(sm.C, Bb, 1);
        __syncthreads();
        double* ur = u + (int64_t)r * N + node1;
#pragma unroll
        for (int q = 0; q < QI; ++q) {
            const int idx = tid + T * q;
            if (idx < NI3) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                ur[ioff[q]] = C(1 + kk, 1 + j, 1 + i);
            }
        }
        __syncthreads();  // the next right-hand side rewrites the cube and the faces
    }
#undef C
}

#define RHS_MB_CASES(X) X(8) X(9) X(10) X(11) X(12)

bool rhs_batched_supported(const Layout& L, int64_t N) {
    return L.NI >= 8 && L.NI <= 12 && N < (int64_t(1) << 32);
}

hipError_t launch_condense_rhs_mb(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                  double* fhat, int k, int R, double* slots, int64_t qlen, hipStream_t st,
                                  SkelStride sk) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    if (ne <= 0 || k <= 0) return hipSuccess;
    if (ne > INT32_MAX || R < 1 || !rhs_batched_supported(g.L, N)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)ne, (unsigned)((k + R - 1) / R));
    switch (g.L.NI) {
#define X(NI)                                                                                                 \
    case NI:                                                                                                  \
        hipLaunchKernelGGL(k_condense_rhs_mb<NI>, grid, dim3(kRhsThreads), 0, st, g, tab, f, N, fhat, k, R, \
                           slots, qlen, sk.ns, sk.rs);                                                        \
        break;
        RHS_MB_CASES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_recover_interior_mb(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                      const double* xskel, double* u, int k, int R, int keep_con, hipStream_t st,
                                      SkelStride sk) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    if (ne <= 0 || k <= 0) return hipSuccess;
    if (ne > INT32_MAX || R < 1 || !rhs_batched_supported(g.L, N)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)ne, (unsigned)((k + R - 1) / R));
    switch (g.L.NI) {
#define X(NI)                                                                                                     \
    case NI:                                                                                                      \
        hipLaunchKernelGGL(k_recover_interior_mb<NI>, grid, dim3(kRhsThreads), 0, st, g, tab, f, N, xskel, u, k, \
                           R, keep_con, sk.ns, sk.rs);                                                            \
        break;
        RHS_MB_CASES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace semcond
