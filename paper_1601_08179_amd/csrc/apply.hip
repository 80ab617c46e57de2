// Condensed Helmholtz operator in the transformed basis: v~ = R H~^_L R^T u~.
//
// Per element (Sec. 6): H~^ = H~_BB - H~_BE D^-1 H~_EB with
//  * primary part H~_BB = restriction to the boundary of
//    d0 M~(x)M~(x)M~ + d1 M~(x)M~(x)K~ + d2 M~(x)K~(x)M~ + d3 K~(x)M~(x)M~, where
//    M~ = diag(M_00, I, M_pp) and K~ has interior block Lambda, boundary entries
//    K_00, K_0p and coupling columns a = S^T K_I0, b = S^T K_Ip (Sec. 6, the
//    transformed mass and stiffness matrices; face self-blocks are diagonal,
//    eq. east_east_primary_part_transformed);
//  * face -> inner eigenspace maps H~_EF of Table 2, e.g. for face w
//    d1 I(x)I(x)K~_I0, which are rank-one along the face normal;
//  * the diagonal D = d0 + d1 Lambda_i + d2 Lambda_j + d3 Lambda_k (eq.
//    hii_diagonal), inverted point-wise;
//  * eigenspace -> face maps H~_FE (Table 2), line reductions along the normal.
// Together 13 n_I^3 multiplications per element for the condensed part
// (Sec. 6) plus O(n_I^2) for the primary part (Table 4).
//
// GPU mapping: one workgroup per element.  The element's 6 faces, 12 edges and
// 8 vertices are gathered (R^T, index arithmetic on the skeleton layout) into
// LDS.  Thread (j,i) owns the column of eigenspace points (k, j, i), k = 0..n_I-1.
// For n_I <= 15 the whole eigenspace vector v = D^-1 u fits in LDS and every
// line reduction is done by the thread owning the output slot; for larger n_I
// the eigenspace is streamed in k-planes (double-buffered), the b/t reductions
// stay in registers and the w/e/s/n line reductions run per plane.  Results
// are summed into the skeleton with hardware floating-point atomics (R).
// Optionally each element's energy u_e . (H~^ u)_e is written, whose sum is
// u . v (used for the CG step length).

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace semcond {

constexpr int apply_threads(int NI) {
    return NI * NI <= 64 ? 64 : ((NI * NI + 63) / 64) * 64;
}

template <typename T, int NI>
__global__ __launch_bounds__(apply_threads(NI)) void k_apply_tpt(ApplyArgs<T> A) {
    constexpr int NI2 = NI * NI;
    constexpr int NT = apply_threads(NI);
    constexpr int NFACE = 6 * NI2;
    constexpr int NSLOT = NFACE + 12 * NI + 8;
    constexpr bool CUBE = NI <= 15;
    constexpr int NW = CUBE ? NI * NI2 : 2 * NI2;

    __shared__ T F[NSLOT];       // gathered u~: faces [6][NI2], edges [12][NI], vertices [8]
    __shared__ T OF[NFACE];      // condensed part of the face outputs
    __shared__ T Wv[NW];         // eigenspace v = D^-1 u (cube or two planes)
    __shared__ T tl[3 * NI];     // Lambda, a, b
    __shared__ int64_t ebase[26];
    __shared__ int econ[26];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int64_t e = (int64_t)blockIdx.x + A.e_begin;
    int e1, e2, e3;
    elem_index(A.g.L, e, &e1, &e2, &e3);
    double dd[4];
    elem_metric(A.g, e, e1, e2, e3, dd);
    const T d0 = (T)dd[0], d1 = (T)dd[1], d2 = (T)dd[2], d3 = (T)dd[3];
    const T m0 = A.tab.m0, K00 = A.tab.K00, K0p = A.tab.K0p;
    const int k = A.k;

    if (tid < 26) {
        bool c;
        element_entity(A.g.L, e1, e2, e3, tid, &ebase[tid], &c);
        econ[tid] = c ? 1 : 0;
    }
    if (tid < NI) {
        tl[tid] = A.tab.lam[tid];
        tl[NI + tid] = A.tab.a[tid];
        tl[2 * NI + tid] = A.tab.b[tid];
    }
    __syncthreads();
    const T* lam = tl;
    const T* ca = tl + NI;
    const T* cb = tl + 2 * NI;

#define UF(f, s1, s2) F[(f) * NI2 + (s1) * NI + (s2)]
#define UE(q, m) F[NFACE + (q) * NI + (m)]
#define UV(q) F[NFACE + 12 * NI + (q)]

    for (int r = 0; r < k; ++r) {
        // ---- gather R^T: skeleton -> element boundary (constrained entities read as 0)
        for (int s = tid; s < NSLOT; s += NT) {
            int ent, loc;
            if (s < NFACE) {
                ent = s / NI2;
                loc = s - ent * NI2;
            } else if (s < NFACE + 12 * NI) {
                int q = (s - NFACE) / NI;
                ent = 6 + q;
                loc = s - NFACE - q * NI;
            } else {
                ent = 18 + (s - NFACE - 12 * NI);
                loc = 0;
            }
            F[s] = econ[ent] ? (T)0 : A.u[(ebase[ent] + loc) * k + r];
        }
        __syncthreads();

        // ---- condensed part: u_E = sum_f H~_EF u_f, v = D^-1 u_E, OF_f = -H~_FE v
        if constexpr (CUBE) {
            if (tid < NI2) {
                const int j = tid / NI, i = tid - (tid / NI) * NI;
                const T ai = ca[i], bi = cb[i], aj = ca[j], bj = cb[j];
                const T Dij = d0 + d1 * lam[i] + d2 * lam[j];
                const T ub = UF(4, j, i), ut = UF(5, j, i);
                T accb = 0, acct = 0;
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) {
                    const T ak = ca[kk], bk = cb[kk];
                    T uc = d1 * (ai * UF(0, kk, j) + bi * UF(1, kk, j)) +
                           d2 * (aj * UF(2, kk, i) + bj * UF(3, kk, i)) + d3 * (ak * ub + bk * ut);
                    T vc = uc * recip<T>(Dij + d3 * lam[kk]);
                    Wv[(kk * NI + j) * NI + i] = vc;
                    accb += ak * vc;
                    acct += bk * vc;
                }
                OF[4 * NI2 + tid] = -d3 * accb;
                OF[5 * NI2 + tid] = -d3 * acct;
            }
            __syncthreads();
            if (tid < NI2) {
                const int s1 = tid / NI, s2 = tid - (tid / NI) * NI;
                T sw = 0, se = 0, ss = 0, sn = 0;
#pragma unroll
                for (int m = 0; m < NI; ++m) {
                    const T vi = Wv[(s1 * NI + s2) * NI + m];  // line along i at (k=s1, j=s2)
                    sw += ca[m] * vi;
                    se += cb[m] * vi;
                    const T vj = Wv[(s1 * NI + m) * NI + s2];  // line along j at (k=s1, i=s2)
                    ss += ca[m] * vj;
                    sn += cb[m] * vj;
                }
                OF[0 * NI2 + tid] = -d1 * sw;
                OF[1 * NI2 + tid] = -d1 * se;
                OF[2 * NI2 + tid] = -d2 * ss;
                OF[3 * NI2 + tid] = -d2 * sn;
            }
        } else {
            const int j = tid / NI, i = tid - (tid / NI) * NI;
            T ai = 0, bi = 0, aj = 0, bj = 0, Dij = 0, ub = 0, ut = 0;
            if (tid < NI2) {
                ai = ca[i];
                bi = cb[i];
                aj = ca[j];
                bj = cb[j];
                Dij = d0 + d1 * lam[i] + d2 * lam[j];
                ub = UF(4, j, i);
                ut = UF(5, j, i);
            }
            T accb = 0, acct = 0;
            for (int kk = 0; kk < NI; ++kk) {
                T* P = Wv + (kk & 1) * NI2;
                if (tid < NI2) {
                    const T ak = ca[kk], bk = cb[kk];
                    T uc = d1 * (ai * UF(0, kk, j) + bi * UF(1, kk, j)) +
                           d2 * (aj * UF(2, kk, i) + bj * UF(3, kk, i)) + d3 * (ak * ub + bk * ut);
                    T vc = uc * recip<T>(Dij + d3 * lam[kk]);
                    P[tid] = vc;
                    accb += ak * vc;
                    acct += bk * vc;
                }
                __syncthreads();
                if (tid < NI) {
                    T sw = 0, se = 0;
                    for (int m = 0; m < NI; ++m) {
                        const T v = P[tid * NI + m];
                        sw += ca[m] * v;
                        se += cb[m] * v;
                    }
                    OF[0 * NI2 + kk * NI + tid] = -d1 * sw;
                    OF[1 * NI2 + kk * NI + tid] = -d1 * se;
                } else if (tid < 2 * NI) {
                    const int c = tid - NI;
                    T ss = 0, sn = 0;
                    for (int m = 0; m < NI; ++m) {
                        const T v = P[m * NI + c];
                        ss += ca[m] * v;
                        sn += cb[m] * v;
                    }
                    OF[2 * NI2 + kk * NI + c] = -d2 * ss;
                    OF[3 * NI2 + kk * NI + c] = -d2 * sn;
                }
            }
            if (tid < NI2) {
                OF[4 * NI2 + tid] = -d3 * accb;
                OF[5 * NI2 + tid] = -d3 * acct;
            }
        }
        __syncthreads();

        // ---- primary part + condensed part, scatter-add R, element energy
        double en = 0.0;
        const T m02 = m0 * m0;
        for (int s = tid; s < NSLOT; s += NT) {
            T out;
            int ent, loc;
            if (s < NFACE) {
                const int f = s / NI2;
                loc = s - f * NI2;
                ent = f;
                const int s1 = loc / NI, s2 = loc - (loc / NI) * NI;
                switch (f) {
                    case 0:  // w: (k, j) = (s1, s2); edges Z(0,0), Z(0,1) along k; Y(0,0), Y(0,1) along j
                        out = (d0 * m0 + d1 * K00 + d2 * m0 * lam[s2] + d3 * m0 * lam[s1]) * UF(0, s1, s2) +
                              d1 * K0p * UF(1, s1, s2) +
                              d2 * m0 * (ca[s2] * UE(8, s1) + cb[s2] * UE(10, s1)) +
                              d3 * m0 * (ca[s1] * UE(4, s2) + cb[s1] * UE(6, s2));
                        break;
                    case 1:  // e
                        out = (d0 * m0 + d1 * K00 + d2 * m0 * lam[s2] + d3 * m0 * lam[s1]) * UF(1, s1, s2) +
                              d1 * K0p * UF(0, s1, s2) +
                              d2 * m0 * (ca[s2] * UE(9, s1) + cb[s2] * UE(11, s1)) +
                              d3 * m0 * (ca[s1] * UE(5, s2) + cb[s1] * UE(7, s2));
                        break;
                    case 2:  // s: (k, i) = (s1, s2); edges Z(0,0), Z(1,0) along k; X(0,0), X(0,1) along i
                        out = (d0 * m0 + d2 * K00 + d1 * m0 * lam[s2] + d3 * m0 * lam[s1]) * UF(2, s1, s2) +
                              d2 * K0p * UF(3, s1, s2) +
                              d1 * m0 * (ca[s2] * UE(8, s1) + cb[s2] * UE(9, s1)) +
                              d3 * m0 * (ca[s1] * UE(0, s2) + cb[s1] * UE(2, s2));
                        break;
                    case 3:  // n
                        out = (d0 * m0 + d2 * K00 + d1 * m0 * lam[s2] + d3 * m0 * lam[s1]) * UF(3, s1, s2) +
                              d2 * K0p * UF(2, s1, s2) +
                              d1 * m0 * (ca[s2] * UE(10, s1) + cb[s2] * UE(11, s1)) +
                              d3 * m0 * (ca[s1] * UE(1, s2) + cb[s1] * UE(3, s2));
                        break;
                    case 4:  // b: (j, i) = (s1, s2); edges Y(0,0), Y(1,0) along j; X(0,0), X(1,0) along i
                        out = (d0 * m0 + d3 * K00 + d1 * m0 * lam[s2] + d2 * m0 * lam[s1]) * UF(4, s1, s2) +
                              d3 * K0p * UF(5, s1, s2) +
                              d1 * m0 * (ca[s2] * UE(4, s1) + cb[s2] * UE(5, s1)) +
                              d2 * m0 * (ca[s1] * UE(0, s2) + cb[s1] * UE(1, s2));
                        break;
                    default:  // t
                        out = (d0 * m0 + d3 * K00 + d1 * m0 * lam[s2] + d2 * m0 * lam[s1]) * UF(5, s1, s2) +
                              d3 * K0p * UF(4, s1, s2) +
                              d1 * m0 * (ca[s2] * UE(6, s1) + cb[s2] * UE(7, s1)) +
                              d2 * m0 * (ca[s1] * UE(2, s2) + cb[s1] * UE(3, s2));
                        break;
                }
                out += OF[s];
            } else if (s < NFACE + 12 * NI) {
                const int q = (s - NFACE) / NI;
                const int m = s - NFACE - q * NI;
                loc = m;
                ent = 6 + q;
                if (q < 4) {  // X(jb,kb) along i: faces b/t (kb) over j, s/n (jb) over k
                    const int jb = q & 1, kb = q >> 1;
                    const T* cj = jb ? cb : ca;
                    const T* ck = kb ? cb : ca;
                    T sf1 = 0, sf2 = 0;
                    for (int m2 = 0; m2 < NI; ++m2) {
                        sf1 += cj[m2] * UF(4 + kb, m2, m);
                        sf2 += ck[m2] * UF(2 + jb, m2, m);
                    }
                    out = (d0 * m02 + d1 * m02 * lam[m] + (d2 + d3) * m0 * K00) * UE(q, m) +
                          d2 * m0 * K0p * UE((1 - jb) + 2 * kb, m) + d3 * m0 * K0p * UE(jb + 2 * (1 - kb), m) +
                          d1 * m02 * (ca[m] * UV(2 * jb + 4 * kb) + cb[m] * UV(1 + 2 * jb + 4 * kb)) +
                          d2 * m0 * sf1 + d3 * m0 * sf2;
                } else if (q < 8) {  // Y(ib,kb) along j: faces b/t (kb) over i, w/e (ib) over k
                    const int ib = (q - 4) & 1, kb = (q - 4) >> 1;
                    const T* ci = ib ? cb : ca;
                    const T* ck = kb ? cb : ca;
                    T sf1 = 0, sf2 = 0;
                    for (int m2 = 0; m2 < NI; ++m2) {
                        sf1 += ci[m2] * UF(4 + kb, m, m2);
                        sf2 += ck[m2] * UF(ib, m2, m);
                    }
                    out = (d0 * m02 + d2 * m02 * lam[m] + (d1 + d3) * m0 * K00) * UE(q, m) +
                          d1 * m0 * K0p * UE(4 + (1 - ib) + 2 * kb, m) + d3 * m0 * K0p * UE(4 + ib + 2 * (1 - kb), m) +
                          d2 * m02 * (ca[m] * UV(ib + 4 * kb) + cb[m] * UV(ib + 2 + 4 * kb)) +
                          d1 * m0 * sf1 + d3 * m0 * sf2;
                } else {  // Z(ib,jb) along k: faces s/n (jb) over i, w/e (ib) over j
                    const int ib = (q - 8) & 1, jb = (q - 8) >> 1;
                    const T* ci = ib ? cb : ca;
                    const T* cj = jb ? cb : ca;
                    T sf1 = 0, sf2 = 0;
                    for (int m2 = 0; m2 < NI; ++m2) {
                        sf1 += ci[m2] * UF(2 + jb, m, m2);
                        sf2 += cj[m2] * UF(ib, m, m2);
                    }
                    out = (d0 * m02 + d3 * m02 * lam[m] + (d1 + d2) * m0 * K00) * UE(q, m) +
                          d1 * m0 * K0p * UE(8 + (1 - ib) + 2 * jb, m) + d2 * m0 * K0p * UE(8 + ib + 2 * (1 - jb), m) +
                          d3 * m02 * (ca[m] * UV(ib + 2 * jb) + cb[m] * UV(ib + 2 * jb + 4)) +
                          d1 * m0 * sf1 + d2 * m0 * sf2;
                }
            } else {
                const int q = s - NFACE - 12 * NI;
                const int ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
                ent = 18 + q;
                loc = 0;
                const T* ci = ib ? cb : ca;
                const T* cj = jb ? cb : ca;
                const T* ck = kb ? cb : ca;
                T sx = 0, sy = 0, sz = 0;
                for (int m2 = 0; m2 < NI; ++m2) {
                    sx += ci[m2] * UE(jb + 2 * kb, m2);
                    sy += cj[m2] * UE(4 + ib + 2 * kb, m2);
                    sz += ck[m2] * UE(8 + ib + 2 * jb, m2);
                }
                out = (d0 * m02 * m0 + (d1 + d2 + d3) * m02 * K00) * UV(q) +
                      m02 * K0p * (d1 * UV(q ^ 1) + d2 * UV(q ^ 2) + d3 * UV(q ^ 4)) +
                      m02 * (d1 * sx + d2 * sy + d3 * sz);
            }
            if (!econ[ent]) {
                atomic_add(&A.v[(ebase[ent] + loc) * k + r], out);
                en += (double)F[s] * (double)out;
            }
        }
        if (A.energy) {
            en = wave_sum(en);
            if ((tid & 63) == 0) red[tid >> 6] = en;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w) s += red[w];
                A.energy[e * k + r] = s;
            }
        }
        __syncthreads();
    }
#undef UF
#undef UE
#undef UV
}

template <typename T>
hipError_t launch_apply_tpt(const ApplyArgs<T>& a, int64_t n_elem, hipStream_t st) {
    const int NI = a.g.L.NI;
    if (n_elem <= 0) return hipSuccess;
    dim3 grid((unsigned)n_elem);
#define CASE(N)                                                                         \
    case N:                                                                             \
        hipLaunchKernelGGL((k_apply_tpt<T, N>), grid, dim3(apply_threads(N)), 0, st, a); \
        break;
    switch (NI) {
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
        CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19)
        CASE(20) CASE(21) CASE(22) CASE(23) CASE(24) CASE(25) CASE(26) CASE(27) CASE(28)
        CASE(29) CASE(30) CASE(31)
        default:
            return hipErrorInvalidValue;
    }
#undef CASE
    return hipGetLastError();
}

template hipError_t launch_apply_tpt<double>(const ApplyArgs<double>&, int64_t, hipStream_t);
template hipError_t launch_apply_tpt<float>(const ApplyArgs<float>&, int64_t, hipStream_t);

}  // namespace semcond
