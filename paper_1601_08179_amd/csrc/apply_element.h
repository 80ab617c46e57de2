// Condensed Helmholtz operator in the transformed basis, v~ = R H~^_L R^T u~:
// per-element device code shared by the standalone apply kernel and the
// persistent CG kernel.
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

#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace semcond {

constexpr int apply_threads(int NI) {
    return NI * NI <= 64 ? 64 : ((NI * NI + 63) / 64) * 64;
}

// Shared memory of one element.
template <typename T, int NI>
struct ApplySmem {
    static constexpr int NI2 = NI * NI;
    static constexpr int NFACE = 6 * NI2;
    static constexpr int NSLOT = NFACE + 12 * NI + 8;
    static constexpr bool CUBE = NI <= 15;
    static constexpr int NW = CUBE ? NI * NI2 : 2 * NI2;
    T F[NSLOT];              // gathered u~: faces [6][NI2], edges [12][NI], vertices [8]
    T OF[CUBE ? 1 : NFACE];  // condensed part of the face outputs (plane mode)
    T Wv[NW];                // eigenspace v = D^-1 u (cube or two planes)
    T tl[3 * NI];            // Lambda, a, b
    int64_t ebase[26];
    int econ[26];
    double red[apply_threads(NI) / 64];
};

// Apply the condensed operator of element e to all k right-hand sides of
// A.u, scattering into A.v.  With DIR the operand is the CG direction
// p = fmadd(beta[r], A.u, A.dir_pinv * A.dir_r), formed at the gather (beta:
// [k], global or shared memory).  The element energies u_e . (H~^ u)_e go to
// A.energy[e*k + r] when A.energy is set and are added to en_acc[r] (shared
// memory, by the group's thread 0) when en_acc is set.  Executed by a group of
// apply_threads(NI) threads with local ids tid; every thread of the workgroup
// must make the same sequence of calls (the function uses workgroup
// barriers).  live = false runs the same code without any global write.
template <typename T, int NI, bool DIR>
__device__ void apply_element(const ApplyArgs<T>& A, int64_t e, ApplySmem<T, NI>& sm, double* en_acc,
                              int tid, bool live, const double* beta) {
    constexpr int NI2 = NI * NI;
    constexpr int NT = apply_threads(NI);
    constexpr int NFACE = 6 * NI2;
    constexpr int NEDGE = 12 * NI;
    constexpr int NSLOT = NFACE + NEDGE + 8;
    constexpr bool CUBE = NI <= 15;
    constexpr int NW = CUBE ? NI * NI2 : 2 * NI2;

    T* const F = sm.F;
    T* const OF = sm.OF;
    T* const Wv = sm.Wv;
    T* const tl = sm.tl;
    int64_t* const ebase = sm.ebase;
    int* const econ = sm.econ;
    double* const red = sm.red;

    int e1, e2, e3;
    elem_index(A.g.L, e, &e1, &e2, &e3);
    double dd[4];
    elem_metric(A.g, e, e1, e2, e3, dd);
    const T d0 = (T)dd[0], d1 = (T)dd[1], d2 = (T)dd[2], d3 = (T)dd[3];
    const T m0 = A.tab.m0, K00 = A.tab.K00, K0p = A.tab.K0p, m02 = m0 * m0;
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
#define UV(q) F[NFACE + NEDGE + (q)]

    for (int r = 0; r < k; ++r) {
        // ---- gather R^T: skeleton -> element boundary (constrained entities read as 0).
        // All loads of a thread are issued before any is consumed: the slot
        // addresses are formed first, constrained slots read index r (a valid
        // node) and are zeroed afterwards.
        {
            constexpr int NG = (NSLOT + NT - 1) / NT;
            int64_t node[NG];
            bool keep[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int s = tid + g * NT;
                int ent = 0, loc = 0;
                if (s < NFACE) {
                    ent = s / NI2;
                    loc = s - ent * NI2;
                } else if (s < NFACE + NEDGE) {
                    const int q = (s - NFACE) / NI;
                    ent = 6 + q;
                    loc = s - NFACE - q * NI;
                } else if (s < NSLOT) {
                    ent = 18 + (s - NFACE - NEDGE);
                }
                keep[g] = s < NSLOT && !econ[ent];
                node[g] = keep[g] ? ebase[ent] + loc : 0;
            }
            T val[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) val[g] = (tid + g * NT < NSLOT) ? A.u[node[g] * k + r] : (T)0;
            if constexpr (DIR) {
                const T bt = (T)beta[r];
                T rv[NG], pv[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const bool in = tid + g * NT < NSLOT;
                    rv[g] = in ? A.dir_r[node[g] * k + r] : (T)0;
                    pv[g] = in ? A.dir_pinv[node[g]] : (T)0;
                }
#pragma unroll
                for (int g = 0; g < NG; ++g) val[g] = fmadd(bt, val[g], pv[g] * rv[g]);
            }
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int s = tid + g * NT;
                if (s < NSLOT) F[s] = keep[g] ? val[g] : (T)0;
            }
        }
        __syncthreads();

        // ---- condensed part: u_E = sum_f H~_EF u_f, v = D^-1 u_E
        if constexpr (CUBE) {
            if (tid < NI2) {
                const int j = tid / NI, i = tid - (tid / NI) * NI;
                const T ai = ca[i], bi = cb[i], aj = ca[j], bj = cb[j];
                const T Dij = d0 + d1 * lam[i] + d2 * lam[j];
                const T ub = UF(4, j, i), ut = UF(5, j, i);
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) {
                    const T uc = d1 * (ai * UF(0, kk, j) + bi * UF(1, kk, j)) +
                                 d2 * (aj * UF(2, kk, i) + bj * UF(3, kk, i)) + d3 * (ca[kk] * ub + cb[kk] * ut);
                    Wv[(kk * NI + j) * NI + i] = uc * recip<T>(Dij + d3 * lam[kk]);
                }
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

        double en = 0.0;
        T* const vr = A.v + r;
        // ---- faces, one algebraic form for all six (Sec. 6 primary part, Table 2
        // condensed part), one face per round so that every face-dependent
        // quantity is wave-uniform.  Face f = w,e,s,n,b,t has slot (s1,s2) =
        // (k,j), (k,j), (k,i), (k,i), (j,i), (j,i); normal / fast / slow axes
        // give d_n, d_fast, d_slow.  Bordering edges (UE index), fast-lo,
        // fast-hi, slow-lo, slow-hi: w {8,10,4,6} e {9,11,5,7} s {8,9,0,2}
        // n {10,11,1,3} b {4,5,0,1} t {6,7,2,3}.
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            constexpr int efl_t[6] = {8, 9, 8, 10, 4, 6}, efh_t[6] = {10, 11, 9, 11, 5, 7};
            constexpr int esl_t[6] = {4, 5, 0, 1, 0, 2}, esh_t[6] = {6, 7, 2, 3, 1, 3};
            const int efl = efl_t[f], efh = efh_t[f], esl = esl_t[f], esh = esh_t[f];
            const T dn = f < 2 ? d1 : (f < 4 ? d2 : d3);
            const T dfast = f < 2 ? d2 : d1;
            const T dslow = f < 4 ? d3 : d2;
            const T* cc = (f & 1) ? cb : ca;
            const bool con = econ[f] != 0;
            const uint32_t fbase = (uint32_t)ebase[f];
            for (int loc = tid; loc < NI2; loc += NT) {
                const int s1 = loc / NI, s2 = loc - (loc / NI) * NI;
                T cond;
                if constexpr (CUBE) {
                    // eigenspace line along the face normal: w/e along i, s/n along j, b/t along k
                    const int base = f < 2 ? loc * NI : (f < 4 ? s1 * NI2 + s2 : loc);
                    constexpr int st_t[3] = {1, NI, NI2};
                    T acc = 0;
#pragma unroll
                    for (int m = 0; m < NI; ++m) acc += cc[m] * Wv[base + m * st_t[f >> 1]];
                    cond = -dn * acc;
                } else {
                    cond = OF[f * NI2 + loc];
                }
                const T uf = F[f * NI2 + loc];
                const T out = (d0 * m0 + dn * K00 + dfast * m0 * lam[s2] + dslow * m0 * lam[s1]) * uf +
                              dn * K0p * F[(f ^ 1) * NI2 + loc] +
                              dfast * m0 * (ca[s2] * UE(efl, s1) + cb[s2] * UE(efh, s1)) +
                              dslow * m0 * (ca[s1] * UE(esl, s2) + cb[s1] * UE(esh, s2)) + cond;
                if (!con && live) {
                    atomic_add(vr + (fbase + (uint32_t)loc) * (uint32_t)k, out);
                    en += (double)uf * (double)out;
                }
            }
        }
        // ---- edges, one direction per round: edge q = 4 par + b0 + 2 b1 along axis
        // `par`, other axes o1, o2 at boundary bits b0, b1.  Neighbour edges differ
        // in one bit; the face couplings are line sums of the two bordering faces.
#pragma unroll
        for (int par = 0; par < 3; ++par) {
            const T dpar = par == 0 ? d1 : (par == 1 ? d2 : d3);
            const T do1 = par == 0 ? d2 : d1;
            const T do2 = par == 2 ? d2 : d3;
            const T dg0 = d0 * m02 + (do1 + do2) * m0 * K00;
            for (int idx = tid; idx < 4 * NI; idx += NT) {
                const int qq = idx / NI, m = idx - (idx / NI) * NI;
                const int b0 = qq & 1, b1 = qq >> 1, q = 4 * par + qq;
                const T* c0 = b0 ? cb : ca;
                const T* c1 = b1 ? cb : ca;
                // X(jb,kb): sum_j c^jb_j b/t(kb)[j][m], sum_k c^kb_k s/n(jb)[k][m]
                // Y(ib,kb): sum_i c^ib_i b/t(kb)[m][i], sum_k c^kb_k w/e(ib)[k][m]
                // Z(ib,jb): sum_i c^ib_i s/n(jb)[m][i], sum_j c^jb_j w/e(ib)[m][j]
                const int f1 = (par == 2 ? 2 : 4) + b1, f2 = (par == 0 ? 2 : 0) + b0;
                const int base1 = f1 * NI2 + (par == 0 ? m : m * NI), st1 = par == 0 ? NI : 1;
                const int base2 = f2 * NI2 + (par == 2 ? m * NI : m), st2 = par == 2 ? 1 : NI;
                T l1 = 0, l2 = 0;
#pragma unroll
                for (int m2 = 0; m2 < NI; ++m2) {
                    l1 += c0[m2] * F[base1 + m2 * st1];
                    l2 += c1[m2] * F[base2 + m2 * st2];
                }
                const int vlo = par == 0 ? 2 * b0 + 4 * b1 : (par == 1 ? b0 + 4 * b1 : b0 + 2 * b1);
                const int vhi = vlo + (par == 0 ? 1 : (par == 1 ? 2 : 4));
                const T ue = UE(q, m);
                const T out = (dg0 + dpar * m02 * lam[m]) * ue + m0 * K0p * (do1 * UE(q ^ 1, m) + do2 * UE(q ^ 2, m)) +
                              dpar * m02 * (ca[m] * UV(vlo) + cb[m] * UV(vhi)) + m0 * (do1 * l1 + do2 * l2);
                if (!econ[6 + q] && live) {
                    atomic_add(vr + ((uint32_t)ebase[6 + q] + (uint32_t)m) * (uint32_t)k, out);
                    en += (double)ue * (double)out;
                }
            }
        }
        // ---- vertices
        if (tid < 8) {
            const int q = tid, ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
            const T* ci_ = ib ? cb : ca;
            const T* cj_ = jb ? cb : ca;
            const T* ck_ = kb ? cb : ca;
            T sx = 0, sy = 0, sz = 0;
#pragma unroll
            for (int m2 = 0; m2 < NI; ++m2) {
                sx += ci_[m2] * UE(jb + 2 * kb, m2);
                sy += cj_[m2] * UE(4 + ib + 2 * kb, m2);
                sz += ck_[m2] * UE(8 + ib + 2 * jb, m2);
            }
            const T out = (d0 * m02 * m0 + (d1 + d2 + d3) * m02 * K00) * UV(q) +
                          m02 * K0p * (d1 * UV(q ^ 1) + d2 * UV(q ^ 2) + d3 * UV(q ^ 4)) +
                          m02 * (d1 * sx + d2 * sy + d3 * sz);
            if (!econ[18 + q] && live) {
                atomic_add(vr + (uint32_t)ebase[18 + q] * (uint32_t)k, out);
                en += (double)UV(q) * (double)out;
            }
        }
        if (A.energy || en_acc) {
            en = wave_sum(en);
            if ((tid & 63) == 0) red[tid >> 6] = en;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int w = 0; w < NT / 64; ++w) sum += red[w];
                if (A.energy && live) A.energy[e * k + r] = sum;
                if (en_acc && live) en_acc[r] += sum;
            }
        }
        __syncthreads();
    }
#undef UF
#undef UE
#undef UV
}

}  // namespace semcond
