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
//    hii_diagonal), inverted point-wise, or in FP32 read from a table of
//    D^-1 per metric class (the paper stores D^-1 per element, Sec. 5);
//  * eigenspace -> face maps H~_FE (Table 2), line reductions along the normal.
// Together 13 n_I^3 multiplications per element for the condensed part
// (Sec. 6) plus O(n_I^2) for the primary part (Sec. 7, the operator-complexity table).
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

#include <type_traits>

#include "cg_device.h"
#include "device_common.h"
#include "kernels.h"

namespace semcond {

constexpr int apply_threads(int NI) {
    return NI * NI <= 64 ? 64 : ((NI * NI + 63) / 64) * 64;
}

// Lanes that one element of the cube body needs: max(n_I^2, 4 n_I, 8) rounded
// up to a power of two; for n_I <= 5 a 64-lane wave then holds several
// elements (apply_pack), one per group of apply_lanes lanes.
constexpr int apply_lanes(int NI) {
    int need = NI * NI > 4 * NI ? NI * NI : 4 * NI;
    if (need < 8) need = 8;
    int l = 8;
    while (l < need) l *= 2;
    return NI <= 5 ? l : apply_threads(NI);
}
constexpr int apply_pack(int NI) { return apply_threads(NI) / apply_lanes(NI); }

// R: the element's row value of a skeleton node, stored into the element's slot
// of the node (qr, the right-hand side's slots, when set; faces only with
// face_slots) or added into vr.
// NS1: a CG apply: node stride 1 (RHS-major vectors) and, with slots, face
// rows in slots exactly in FP32 (the launcher checks both).
template <bool SL = true, bool NS1 = false, typename T>
__device__ inline void out_store(const ApplyArgs<T>& A, T* vr, T* qr, uint32_t node, int slot, T val,
                                 bool face = false) {
    const bool fslots = NS1 ? sizeof(T) == 4 : A.face_slots != 0;
    if constexpr (NS1) {
        // 32-bit byte offsets from the right-hand side's uniform bases (a
        // slot offset is below 2 N_s + 6 (N_s - oV), N_s sizeof(T) < 2^31)
        if (SL && qr && (!face || fslots))
            *(T*)((char*)qr + slot_addr(A.g.L, node, slot) * (uint32_t)sizeof(T)) = val;
        else
            atomic_add((T*)((char*)vr + node * (uint32_t)sizeof(T)), val);
    } else {
        if (SL && qr && (!face || fslots))
            qr[slot_addr(A.g.L, node, slot)] = val;
        else
            atomic_add(vr + node * A.ns, val);
    }
}

// Shared memory of one element.
template <typename T, int NI>
struct ApplySmem {
    static constexpr int NI2 = NI * NI;
    static constexpr int NFACE = 6 * NI2;
    static constexpr int NSLOT = NFACE + 12 * NI + 8;
    static constexpr bool CUBE = NI <= 15;
    static constexpr int NW = CUBE ? NI * NI2 : 2 * NI2;
    // the 1D coefficients first: at small LDS addresses their pairs are read
    // with immediate offsets from one zero base (ds_read2 offsets reach 255 elements)
    T tl[3 * NI];            // Lambda, a, b
    T F[NSLOT];              // gathered u~: faces [6][NI2], edges [12][NI], vertices [8]
    T OF[CUBE ? 1 : NFACE];  // condensed part of the face outputs (plane mode)
    T Wv[NW];                // eigenspace v = D^-1 u (cube or two planes)
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
__device__ void apply_element_planes(const ApplyArgs<T>& A, int64_t e, ApplySmem<T, NI>& sm, double* en_acc,
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
    const T d0e = (T)dd[0], d1e = (T)dd[1], d2e = (T)dd[2], d3e = (T)dd[3];
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
    // line-sum split of the plane path: RG lanes per line (largest power of
    // two <= 16 with all 2 n_I lines in one round), RT terms per lane
    constexpr int RG = 2 * NI * 16 <= NT ? 16 : (2 * NI * 8 <= NT ? 8 : 4);
    constexpr int RT = (NI + RG - 1) / RG;
    const int rh = tid & (RG - 1);
    T rca[RT], rcb[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int m = rh + RG * q;
        rca[q] = m < NI ? ca[m] : (T)0;
        rcb[q] = m < NI ? cb[m] : (T)0;
    }

#define UF(f, s1, s2) F[(f) * NI2 + (s1) * NI + (s2)]
#define UE(q, m) F[NFACE + (q) * NI + (m)]
#define UV(q) F[NFACE + NEDGE + (q)]

    for (int r = 0; r < k; ++r) {
        if (A.act && !A.act[r]) continue;  // a stopped right-hand side
        // The products of the metric terms are formed anew for every right-hand
        // side instead of being kept live across the loop (register pressure).
        T d0 = d0e, d1 = d1e, d2 = d2e, d3 = d3e;
        asm volatile("" : "+v"(d0), "+v"(d1), "+v"(d2), "+v"(d3));
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
                keep[g] = s < NSLOT && (!econ[ent] || A.read_con);
                node[g] = keep[g] ? ebase[ent] + loc : 0;
            }
            T val[NG];
            const uint32_t ns = DIR ? 1u : A.ns;  // CG directions are RHS-major
#pragma unroll
            for (int g = 0; g < NG; ++g) val[g] = (tid + g * NT < NSLOT) ? A.u[node[g] * ns + r * A.rs] : (T)0;
            if constexpr (DIR) {
                const T bt = (T)beta[r];
                T rv[NG], pv[NG];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const bool in = tid + g * NT < NSLOT;
                    rv[g] = in ? A.dir_r[node[g] + r * A.rs] : (T)0;
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
                // Line sums of the plane (Table 2): w/e along i for row j = l,
                // s/n along j for column i = l, with both coefficient rows.
                // Each line takes an aligned group of RG lanes, lane h summing
                // the terms h, h + RG, ... with its preloaded coefficients; the
                // group's partial sums are combined by a fixed in-row tree.
                for (int line = tid / RG; line < 2 * NI; line += NT / RG) {
                    const bool row = line < NI;
                    const int l = row ? line : line - NI;
                    const int sl = row ? NI : 1, sm = row ? 1 : NI;
                    T sa = 0, sb = 0;
#pragma unroll
                    for (int q = 0; q < RT; ++q) {
                        const int m = rh + RG * q;
                        const T v = m < NI ? P[l * sl + m * sm] : (T)0;
                        sa += rca[q] * v;
                        sb += rcb[q] * v;
                    }
                    sa = group_sum<RG>(sa);
                    sb = group_sum<RG>(sb);
                    if (rh == 0) {
                        const T dl = row ? -d1 : -d2;
                        const int o = (row ? 0 : 2) * NI2 + kk * NI + l;
                        OF[o] = dl * sa;
                        OF[o + NI2] = dl * sb;
                    }
                }
            }
            if (tid < NI2) {
                OF[4 * NI2 + tid] = -d3 * accb;
                OF[5 * NI2 + tid] = -d3 * acct;
            }
        }
        __syncthreads();

        double en = 0.0;
        T* const vr = A.v + (size_t)r * A.rs;
        T* const qr = A.slots ? A.slots + (size_t)r * A.qlen : nullptr;
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
                    out_store<true, DIR>(A, vr, qr, fbase + (uint32_t)loc, 1 - (f & 1), out, true);
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
                // X(jb,kb): sum_j c^jb_j b/t(kb)[j][m], sum_k c^kb_k s/n(jb)[k][m]
                // Y(ib,kb): sum_i c^ib_i b/t(kb)[m][i], sum_k c^kb_k w/e(ib)[k][m]
                // Z(ib,jb): sum_i c^ib_i s/n(jb)[m][i], sum_j c^jb_j w/e(ib)[m][j]
                const int f1 = (par == 2 ? 2 : 4) + b1, f2 = (par == 0 ? 2 : 0) + b0;
                const int base1 = f1 * NI2 + (par == 0 ? m : m * NI), st1 = par == 0 ? NI : 1;
                const int base2 = f2 * NI2 + (par == 2 ? m * NI : m), st2 = par == 2 ? 1 : NI;
                // both coefficient rows, then the thread's pick (no per-term selects)
                T l1a = 0, l1b = 0, l2a = 0, l2b = 0;
#pragma unroll 2
                for (int m2 = 0; m2 < NI; ++m2) {
                    const T am = ca[m2], bm = cb[m2];
                    const T x1 = F[base1 + m2 * st1], x2 = F[base2 + m2 * st2];
                    l1a += am * x1;
                    l1b += bm * x1;
                    l2a += am * x2;
                    l2b += bm * x2;
                }
                const T l1 = b0 ? l1b : l1a, l2 = b1 ? l2b : l2a;
                const int vlo = par == 0 ? 2 * b0 + 4 * b1 : (par == 1 ? b0 + 4 * b1 : b0 + 2 * b1);
                const int vhi = vlo + (par == 0 ? 1 : (par == 1 ? 2 : 4));
                const T ue = UE(q, m);
                const T out = (dg0 + dpar * m02 * lam[m]) * ue + m0 * K0p * (do1 * UE(q ^ 1, m) + do2 * UE(q ^ 2, m)) +
                              dpar * m02 * (ca[m] * UV(vlo) + cb[m] * UV(vhi)) + m0 * (do1 * l1 + do2 * l2);
                if (!econ[6 + q] && live) {
                    out_store<true, DIR>(A, vr, qr, (uint32_t)ebase[6 + q] + (uint32_t)m, (1 - b0) + 2 * (1 - b1), out);
                    en += (double)ue * (double)out;
                }
            }
        }
        // ---- vertices
        if (tid < 8) {
            const int q = tid, ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
            T sxa = 0, sxb = 0, sya = 0, syb = 0, sza = 0, szb = 0;
#pragma unroll 2
            for (int m2 = 0; m2 < NI; ++m2) {
                const T am = ca[m2], bm = cb[m2];
                const T x = UE(jb + 2 * kb, m2), y = UE(4 + ib + 2 * kb, m2), z = UE(8 + ib + 2 * jb, m2);
                sxa += am * x;
                sxb += bm * x;
                sya += am * y;
                syb += bm * y;
                sza += am * z;
                szb += bm * z;
            }
            const T sx = ib ? sxb : sxa, sy = jb ? syb : sya, sz = kb ? szb : sza;
            const T out = (d0 * m02 * m0 + (d1 + d2 + d3) * m02 * K00) * UV(q) +
                          m02 * K0p * (d1 * UV(q ^ 1) + d2 * UV(q ^ 2) + d3 * UV(q ^ 4)) +
                          m02 * (d1 * sx + d2 * sy + d3 * sz);
            if (!econ[18 + q] && live) {
                out_store<true, DIR>(A, vr, qr, (uint32_t)ebase[18 + q], (1 - ib) + 2 * (1 - jb) + 4 * (1 - kb), out);
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

// Wave-uniform skeleton entities of element (e1,e2,e3): face bases (w, e, s,
// n, b, t), edge bases of the three directions at boundary bits (0, 0), the
// vertex base, and the Dirichlet flags of the element's six boundary planes.
// [N_s][k] offsets stay below 2^31, so node indices are 32-bit.
struct ElemEnt {
    uint32_t fb[6];
    uint32_t eb[3];
    uint32_t vb;
    bool cx0, cx1, cy0, cy1, cz0, cz1;
};

__device__ inline void elem_entities(const Layout& L, int e1, int e2, int e3, ElemEnt& E) {
    E.fb[0] = (uint32_t)fx_base(L, e3, e2, e1);
    E.fb[1] = (uint32_t)fx_base(L, e3, e2, e1 + 1);
    E.fb[2] = (uint32_t)fy_base(L, e3, e2, e1);
    E.fb[3] = (uint32_t)fy_base(L, e3, e2 + 1, e1);
    E.fb[4] = (uint32_t)fz_base(L, e3, e2, e1);
    E.fb[5] = (uint32_t)fz_base(L, e3 + 1, e2, e1);
    E.eb[0] = (uint32_t)ex_base(L, e3, e2, e1);
    E.eb[1] = (uint32_t)ey_base(L, e3, e2, e1);
    E.eb[2] = (uint32_t)ez_base(L, e3, e2, e1);
    E.vb = (uint32_t)v_base(L, e3, e2, e1);
    E.cx0 = xcon(L, e1);
    E.cx1 = xcon(L, e1 + 1);
    E.cy0 = ycon(L, e2);
    E.cy1 = ycon(L, e2 + 1);
    E.cz0 = zcon(L, e3);
    E.cz1 = zcon(L, e3 + 1);
}

// Node and Dirichlet flag of the thread's edge node in direction par (edge
// X(jb,kb), Y(ib,kb), Z(ib,jb) with bits (b0, b1), node m) and of its vertex
// (ib, jb, kb).
template <int NI>
__device__ inline void edge_node(const Layout& L, const ElemEnt& E, int par, int b0, int b1, int m, uint32_t* node,
                                 bool* con) {
    const uint32_t n1 = (uint32_t)L.n1, n2 = (uint32_t)L.n2;
    const uint32_t s0 = par == 0 ? n1 * NI : (uint32_t)NI;
    const uint32_t s1 = par == 0 ? (n2 + 1) * n1 * NI : (par == 1 ? n2 * (n1 + 1) * NI : (n1 + 1) * NI);
    *node = E.eb[par] + (b0 ? s0 : 0u) + (b1 ? s1 : 0u) + m;
    const bool c0 = par == 0 ? (b0 ? E.cy1 : E.cy0) : (b0 ? E.cx1 : E.cx0);
    const bool c1 = par == 2 ? (b1 ? E.cy1 : E.cy0) : (b1 ? E.cz1 : E.cz0);
    *con = c0 || c1;
}
__device__ inline void vertex_node(const Layout& L, const ElemEnt& E, int ib, int jb, int kb, uint32_t* node,
                                   bool* con) {
    const uint32_t n1 = (uint32_t)L.n1, n2 = (uint32_t)L.n2;
    *node = E.vb + ib + (jb ? n1 + 1 : 0u) + (kb ? (n2 + 1) * (n1 + 1) : 0u);
    *con = (ib ? E.cx1 : E.cx0) || (jb ? E.cy1 : E.cy0) || (kb ? E.cz1 : E.cz0);
}

// One thread's gathered values of one (element, RHS): its face slot of the
// six faces, its edge node in the three directions, its vertex.  With DIR
// also r and P^-1 at the same nodes.  Constrained slots hold 0 (DIR: zero
// directions), slots the thread does not own an unspecified value.
template <typename T, bool DIR>
struct Gathered {
    T f[6], e[3], v;
    T rf[6], re[3], rv;
    T pf[6], pe[3], pv;
};

// Issue the loads of item (e, r); nothing is waited for here.  Edge node
// (edge te / n_I, node te mod n_I) is lane te + ESHIFT's.
template <typename T, int NI, bool DIR, int ESHIFT = 0>
__device__ inline void gather_issue(const ApplyArgs<T>& A, int64_t e, bool live, uint32_t r, int t,
                                    Gathered<T, DIR>& G) {
    constexpr int NI2 = NI * NI;
    const Layout& L = A.g.L;
    int e1, e2, e3;
    elem_index(L, live ? e : 0, &e1, &e2, &e3);
    ElemEnt E;
    elem_entities(L, e1, e2, e3, E);
    const bool fcon[6] = {E.cx0, E.cx1, E.cy0, E.cy1, E.cz0, E.cz1};
    // CG directions (DIR) are RHS-major (node stride 1): the right-hand side's
    // vectors start at wave-uniform addresses and a node is a 32-bit byte
    // offset from them (N_s sizeof(T) < 2^32, checked by the launcher), which
    // the loads take as a vector offset from a scalar base.
    const char* const ub = DIR ? (const char*)(A.u + (size_t)r * A.rs) : nullptr;
    const char* const rb = DIR ? (const char*)(A.dir_r + (size_t)r * A.rs) : nullptr;
    const char* const pb = DIR ? (const char*)A.dir_pinv : nullptr;
    // own: the lane owns the node; con: the node is constrained.  A CG
    // direction is zero at constrained nodes by itself (P^-1 and the previous
    // direction are zero there: every direction is formed as beta p + P^-1 r
    // from a zero start), so DIR lanes load every node they own and leave the
    // others' values unset (never read: the commit writes owned nodes only);
    // plain applies read constrained nodes as 0 unless read_con.
    // Packed elements (n_I <= 5, several per wave) index the vectors by
    // element instead of by byte offset: measured 4 % faster there.
    auto load = [&](uint32_t node, bool own, bool con, T& u, T& rr, T& pp) {
        if constexpr (DIR) {
            u = __builtin_nondeterministic_value(u);
            rr = __builtin_nondeterministic_value(rr);
            pp = __builtin_nondeterministic_value(pp);
            if (own) {
                if constexpr (NI > 5) {
                    const uint32_t bo = node * (uint32_t)sizeof(T);
                    u = *(const T*)(ub + bo);
                    rr = *(const T*)(rb + bo);
                    pp = *(const T*)(pb + bo);
                } else {
                    const uint32_t off = node + r * A.rs;
                    u = A.u[off];
                    rr = A.dir_r[off];
                    pp = A.dir_pinv[node];
                }
            }
        } else {
            u = (T)0;
            if (own && (!con || A.read_con)) u = A.u[node * A.ns + r * A.rs];
        }
    };
    const bool fown = live && t < NI2;
#pragma unroll
    for (int f = 0; f < 6; ++f) load(E.fb[f] + (uint32_t)t, fown, fcon[f], G.f[f], G.rf[f], G.pf[f]);
    const int te = t - ESHIFT, tq = te >= 0 ? te : 0;
    const int eq = tq / NI, em = tq - (tq / NI) * NI;
    const bool eown = live && te >= 0 && te < 4 * NI;
#pragma unroll
    for (int par = 0; par < 3; ++par) {
        uint32_t node;
        bool con;
        edge_node<NI>(L, E, par, eq & 1, (eq >> 1) & 1, em, &node, &con);
        load(node, eown, con, G.e[par], G.re[par], G.pe[par]);
    }
    {
        uint32_t node;
        bool con;
        vertex_node(L, E, t & 1, (t >> 1) & 1, (t >> 2) & 1, &node, &con);
        load(node, live && t < 8, con, G.v, G.rv, G.pv);
    }
}

// Element body for n_I <= 15: the eigenspace cube lives in LDS.  Entity bases
// and Dirichlet flags are wave-uniform (scalar) values; the 1D coefficients at
// a uniform index come from the launch arguments.  Thread t < n_I^2 owns the
// face slot (s1, s2) = (t / n_I, t mod n_I) of every face and the eigenspace
// column (k, s1, s2), k = 0..n_I-1; thread t < 4 n_I owns edge node t mod n_I
// of edge t / n_I of each direction; thread t < 8 owns vertex t.
// With ONE the group computes the single item (element e0, RHS r0) (e0 at or
// beyond n_end: without global writes); otherwise it walks `count` elements
// e0, e0 + stride, ... and for each the right-hand sides r0 .. r0 + nr - 1.  (A
// loop keeps the coefficient scalars live across items; the single-item form
// lets them live only where they are used.)
// With NE > 1 (ONE only) the workgroup holds NE groups of NT / NE lanes; group g
// computes element e0 + g with its own LDS block smv[g].
template <typename T, int NI, bool DIR, bool ONE, int NE = 1, bool FZ = false>
__device__ void apply_elements_cube(const ApplyArgs<T>& A, int64_t e0, int64_t stride, int64_t count, int64_t n_end,
                                    uint32_t r0, uint32_t nr, ApplySmem<T, NI>* smv, double* en_acc, int tid,
                                    const double* beta) {
    static_assert(NE == 1 || ONE, "packed elements only in the single-item form");
    constexpr int NI2 = NI * NI;
    constexpr int NT = apply_threads(NI) / NE;  // lanes per element
    constexpr int NFACE = 6 * NI2;
    constexpr int NEDGE = 12 * NI;
    const int grp = NE == 1 ? 0 : tid / NT;
    ApplySmem<T, NI>& sm = smv[grp];
    T* const F = sm.F;
    T* const Wv = sm.Wv;
    double* const red = sm.red;
    const Layout& L = A.g.L;
    const int t = NE == 1 ? tid : tid - grp * NT;
    const uint32_t k = (uint32_t)A.k;
    const T m0 = A.tab.m0, K00 = A.tab.K00, K0p = A.tab.K0p, m02 = m0 * m0;

    // per-thread position and 1D coefficients of the face slot (s1 slow, s2 fast),
    // edge node and vertex: the same for every element.  With several waves
    // the edge nodes go to the last wave (lanes NT - 64 ..), which holds the
    // fewest face slots, and the vertices stay in the first: the waves' row
    // work is then closer to even (they meet at the energy barrier).  Measured
    // faster in FP32 (CG apply at n_I = 11, 16 RHS: 4.6 %), in the fused FP64
    // CG kernels, in the other FP64 CG applies except at n_I = 11 (16-RHS
    // solves 2.5-4 % faster at n_I = 9, 10, 12, 13) and in the plain FP64
    // applies at n_I >= 12; slower in the plain FP64 applies at n_I = 9..11
    // and in the FP64 CG apply at n_I = 11 (3-5 %), whose edge rounds sum both
    // coefficient rows.
    static_assert(4 * NI <= 64, "the edge nodes of one direction fit one wave");
    constexpr int ESHIFT =
        NE == 1 && NT >= 128 && (sizeof(T) == 4 || FZ || (NI != 11 && (DIR || NI >= 12))) ? NT - 64 : 0;
    const int te = t - ESHIFT, tq = te >= 0 ? te : 0;
    const bool fown = t < NI2, eown = te >= 0 && te < 4 * NI, vown = t < 8;
    const int s1 = t / NI, s2 = t - (t / NI) * NI;
    const int eq = tq / NI, em = tq - (tq / NI) * NI;  // edge qq = b0 + 2 b1, node m
    const int eb0 = eq & 1, eb1 = (eq >> 1) & 1;
    const int vib = t & 1, vjb = (t >> 1) & 1, vkb = (t >> 2) & 1;
    T ta1 = 0, tb1 = 0, tl1 = 0, ta2 = 0, tb2 = 0, tl2 = 0;
    if (fown || eown) {
        ta1 = A.tab.a[s1 < NI ? s1 : 0];
        tb1 = A.tab.b[s1 < NI ? s1 : 0];
        tl1 = A.tab.lam[s1 < NI ? s1 : 0];
        ta2 = A.tab.a[s2];
        tb2 = A.tab.b[s2];
        tl2 = A.tab.lam[s2];
    }

#define UE(q, m) F[NFACE + (q) * NI + (m)]
#define UV(q) F[NFACE + NEDGE + (q)]

    // the 1D coefficients at wave-uniform indices: an LDS copy (broadcast reads)
    T* const ctL = sm.tl;
    T* const ctA = sm.tl + NI;
    T* const ctB = sm.tl + 2 * NI;
    if (t < NI) {
        ctL[t] = A.tab.lam[t];
        ctA[t] = A.tab.a[t];
        ctB[t] = A.tab.b[t];
    }  // read after the first item's gather barrier

    // fused completion of the previous CG step's r.z (single-item form): the
    // workgroup's threads reduce the step's partial sums while the gather's
    // loads are in flight
    constexpr int WG = apply_threads(NI);
    __shared__ double s_fz[FZ ? 2 * (WG / 64) : 1];

    auto item = [&](const int64_t e, const bool live, const uint32_t r) __attribute__((always_inline)) {
        // a stopped right-hand side (the same in the whole workgroup); only the CG
        // loop with separate reductions passes activity flags, and slots only it
        // and the deterministic plain applies
        constexpr bool SL = !FZ;
        if constexpr (SL) {
            if (A.act && !A.act[r]) return;
        }
        if constexpr (DIR && ONE && FZ) {
            if (!A.fz.act_prev[r]) {  // stopped before this iteration: nothing to gather
                if (blockIdx.x == 0 && tid == 0) cg_carry_stopped(A.fz, (int)r);
                return;
            }
        }
        Gathered<T, DIR> G;
        gather_issue<T, NI, DIR, ESHIFT>(A, e, live, r, t, G);
        // FP32: the thread's D^-1 column from its metric class's table (one
        // class per workgroup: single-element groups only), loaded with the
        // gather.  The table holds 1/D rounded once from FP64, which the FP32
        // CG converges with measurably fewer iterations than with D inverted
        // in FP32; FP64 keeps the point-wise inverse (measured faster there),
        // and so do the fused CG kernels (FZ), whose registers are at a limit.
        constexpr bool TAB = sizeof(T) == 4 && NE == 1 && !FZ;
        const bool use_tab = TAB && A.dinv != nullptr;
        T dvr[TAB ? NI : 1];
        if constexpr (TAB) {
            if (use_tab && fown) {
                const T* dtab = A.dinv + (size_t)(A.dcls ? A.dcls[live ? e : 0] : 0) * (NI * NI2) + t;
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) dvr[kk] = dtab[kk * NI2];
            }
        }
        T bt = DIR ? (T)beta[r] : (T)0;
        if constexpr (DIR && ONE && FZ) {
            {
                double sums[2];
                block_sums<WG, 2, (NI <= 5 ? 2 : 4)>(A.fz.part + r, (int64_t)A.fz.nsb * A.k, A.fz.nsb, A.k, s_fz, sums);
                bool still;
                bt = (T)cg_rz_complete(A.fz, (int)r, sums[0], sums[1], blockIdx.x == 0 && tid == 0, &still);
                // a stopped RHS is not applied (the step ignores its energies)
                if (!still) return;
            }
        }
        // ---- commit the gathered values (R^T) to LDS
        {
            auto val = [&](T u, T rr, T pp) -> T {
                if constexpr (DIR) return fmadd(bt, u, pp * rr);
                return u;
            };
            if (fown) {
#pragma unroll
                for (int f = 0; f < 6; ++f) F[f * NI2 + t] = val(G.f[f], G.rf[f], G.pf[f]);
            }
            if (eown) {
#pragma unroll
                for (int par = 0; par < 3; ++par) F[NFACE + par * 4 * NI + te] = val(G.e[par], G.re[par], G.pe[par]);
            }
            if (vown) UV(t) = val(G.v, G.rv, G.pv);
        }
        __syncthreads();

        int e1, e2, e3;
        elem_index(L, live ? e : 0, &e1, &e2, &e3);
        double dd[4];
        elem_metric(A.g, live ? e : 0, e1, e2, e3, dd);
        const T d0 = (T)dd[0], d1 = (T)dd[1], d2 = (T)dd[2], d3 = (T)dd[3];
        ElemEnt E;
        elem_entities(L, e1, e2, e3, E);
        const bool fcon[6] = {E.cx0, E.cx1, E.cy0, E.cy1, E.cz0, E.cz1};

        // ---- condensed part (Table 2): v = D^-1 sum_f H~_EF u_f on column (k, s1, s2);
        // the b/t line reductions along k stay in registers.
        T accb = 0, acct = 0;
        if (fown) {
            const T Dij = d0 + d1 * tl2 + d2 * tl1;
            const T wa = d1 * ta2, wb = d1 * tb2, sa = d2 * ta1, sb = d2 * tb1;
            const T ub = d3 * F[4 * NI2 + t], ut = d3 * F[5 * NI2 + t];
            auto column = [&](auto use_table) __attribute__((always_inline)) {
#pragma unroll
                for (int kk = 0; kk < NI; ++kk) {
                    const T ak = ctA[kk], bk = ctB[kk];
                    const T uc = wa * F[kk * NI + s1] + wb * F[NI2 + kk * NI + s1] + sa * F[2 * NI2 + kk * NI + s2] +
                                 sb * F[3 * NI2 + kk * NI + s2] + ak * ub + bk * ut;
                    T dv;
                    if constexpr (decltype(use_table)::value)
                        dv = dvr[kk];
                    else
                        dv = recip<T>(Dij + d3 * ctL[kk]);
                    const T v = uc * dv;
                    Wv[kk * NI2 + t] = v;
                    accb += ak * v;
                    acct += bk * v;
                }
            };
            if constexpr (TAB) {
                if (use_tab)
                    column(std::integral_constant<bool, true>{});
                else
                    column(std::integral_constant<bool, false>{});
            } else {
                column(std::integral_constant<bool, false>{});
            }
        }
        __syncthreads();

        double en = 0.0;
        T* const vr = A.v + (size_t)r * A.rs;
        T* const qr = SL && A.slots ? A.slots + (size_t)r * A.qlen : nullptr;
        // ---- faces: primary part (Sec. 6) + condensed part (Table 2), pairs w/e, s/n, b/t.
        // Face f has slots (k,j), (k,j), (k,i), (k,i), (j,i), (j,i); bordering edges (UE index)
        // fast-lo, fast-hi, slow-lo, slow-hi: w {8,10,4,6} e {9,11,5,7} s {8,9,0,2}
        // n {10,11,1,3} b {4,5,0,1} t {6,7,2,3}.
        if (fown) {
            T cnd[6];
            {
                T sw = 0, se = 0, ss = 0, sn = 0;
#pragma unroll
                for (int m = 0; m < NI; ++m) {
                    const T vw = Wv[t * NI + m];              // line along i at (k, j) = (s1, s2)
                    const T vs = Wv[s1 * NI2 + m * NI + s2];  // line along j at (k, i) = (s1, s2)
                    const T am = ctA[m], bm = ctB[m];
                    sw += am * vw;
                    se += bm * vw;
                    ss += am * vs;
                    sn += bm * vs;
                }
                cnd[0] = -d1 * sw;
                cnd[1] = -d1 * se;
                cnd[2] = -d2 * ss;
                cnd[3] = -d2 * sn;
                cnd[4] = -d3 * accb;
                cnd[5] = -d3 * acct;
            }
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                constexpr int efl_t[6] = {8, 9, 8, 10, 4, 6}, efh_t[6] = {10, 11, 9, 11, 5, 7};
                constexpr int esl_t[6] = {4, 5, 0, 1, 0, 2}, esh_t[6] = {6, 7, 2, 3, 1, 3};
                const T dn = f < 2 ? d1 : (f < 4 ? d2 : d3);
                const T dfast = f < 2 ? d2 : d1;
                const T dslow = f < 4 ? d3 : d2;
                const T uf = F[f * NI2 + t];
                const T out = (d0 * m0 + dn * K00 + dfast * m0 * tl2 + dslow * m0 * tl1) * uf +
                              dn * K0p * F[(f ^ 1) * NI2 + t] +
                              dfast * m0 * (ta2 * UE(efl_t[f], s1) + tb2 * UE(efh_t[f], s1)) +
                              dslow * m0 * (ta1 * UE(esl_t[f], s2) + tb1 * UE(esh_t[f], s2)) + cnd[f];
                if (!fcon[f] && live) {
                    out_store<SL, DIR && (NI > 5)>(A, vr, qr, E.fb[f] + (uint32_t)t, 1 - (f & 1), out, true);
                    en += (double)uf * (double)out;
                }
            }
        }
        // ---- edges, one direction per round: edge q = 4 par + b0 + 2 b1; the face
        // couplings are line sums of the two bordering faces.
        if (eown) {
            // the 1D coefficients at the edge node m: ta2, tb2, tl2 where the
            // edge and face lanes coincide, else from the LDS copy
            T tae = ta2, tbe = tb2, tle = tl2;
            if constexpr (ESHIFT > 0) {
                tae = ctA[em];
                tbe = ctB[em];
                tle = ctL[em];
            }
            // FP32: the thread's two coefficient rows (c^eb0, c^eb1: the same
            // edge bits in every direction), picked once for the three rounds;
            // FP64 sums both rows and picks (measured 11 % faster there: the
            // picked rows hold 44 more VGPRs through the rounds)
            constexpr bool ROWS = sizeof(T) == 4;
            T c1r[ROWS ? NI : 1], c2r[ROWS ? NI : 1];
            if constexpr (ROWS) {
#pragma unroll
                for (int m2 = 0; m2 < NI; ++m2) {
                    const T am = ctA[m2], bm = ctB[m2];
                    c1r[m2] = eb0 ? bm : am;
                    c2r[m2] = eb1 ? bm : am;
                }
            }
#pragma unroll
            for (int par = 0; par < 3; ++par) {
                const T dpar = par == 0 ? d1 : (par == 1 ? d2 : d3);
                const T do1 = par == 0 ? d2 : d1;
                const T do2 = par == 2 ? d2 : d3;
                const T dg0 = d0 * m02 + (do1 + do2) * m0 * K00;
                const int q = 4 * par + eq;
                // X(jb,kb): sum_j c^jb_j b/t(kb)[j][m], sum_k c^kb_k s/n(jb)[k][m]
                // Y(ib,kb): sum_i c^ib_i b/t(kb)[m][i], sum_k c^kb_k w/e(ib)[k][m]
                // Z(ib,jb): sum_i c^ib_i s/n(jb)[m][i], sum_j c^jb_j w/e(ib)[m][j]
                const int f1 = (par == 2 ? 2 : 4) + eb1, f2 = (par == 0 ? 2 : 0) + eb0;
                const int base1 = f1 * NI2 + (par == 0 ? em : em * NI);
                const int base2 = f2 * NI2 + (par == 2 ? em * NI : em);
                constexpr int st1_t[3] = {NI, 1, 1}, st2_t[3] = {NI, NI, 1};
                T l1 = 0, l2 = 0;
                if constexpr (ROWS) {
#pragma unroll
                    for (int m2 = 0; m2 < NI; ++m2) {
                        l1 += c1r[m2] * F[base1 + m2 * st1_t[par]];
                        l2 += c2r[m2] * F[base2 + m2 * st2_t[par]];
                    }
                } else {
                    T l1a = 0, l1b = 0, l2a = 0, l2b = 0;
#pragma unroll
                    for (int m2 = 0; m2 < NI; ++m2) {
                        const T am = ctA[m2], bm = ctB[m2];
                        const T x1 = F[base1 + m2 * st1_t[par]], x2 = F[base2 + m2 * st2_t[par]];
                        l1a += am * x1;
                        l1b += bm * x1;
                        l2a += am * x2;
                        l2b += bm * x2;
                    }
                    l1 = eb0 ? l1b : l1a;
                    l2 = eb1 ? l2b : l2a;
                }
                const int vlo = par == 0 ? 2 * eb0 + 4 * eb1 : (par == 1 ? eb0 + 4 * eb1 : eb0 + 2 * eb1);
                const int vhi = vlo + (par == 0 ? 1 : (par == 1 ? 2 : 4));
                const T ue = UE(q, em);
                const T out = (dg0 + dpar * m02 * tle) * ue + m0 * K0p * (do1 * UE(q ^ 1, em) + do2 * UE(q ^ 2, em)) +
                              dpar * m02 * (tae * UV(vlo) + tbe * UV(vhi)) + m0 * (do1 * l1 + do2 * l2);
                uint32_t node;
                bool con;
                edge_node<NI>(L, E, par, eb0, eb1, em, &node, &con);
                if (!con && live) {
                    out_store<SL, DIR && (NI > 5)>(A, vr, qr, node, (1 - eb0) + 2 * (1 - eb1), out);
                    en += (double)ue * (double)out;
                }
            }
        }
        // ---- vertices: the couplings to the three edges through a vertex are
        // line sums along those edges.  In FP32 with a whole wave at hand the
        // 24 sums (8 vertices x 3 directions) run on 24 lanes and every vertex
        // lane collects its three; otherwise (FP64: measured faster; packed
        // elements, n_I <= 5) each vertex lane sums all three.
        constexpr bool VLANES = sizeof(T) == 4 && NE == 1 && NT >= 64;
        T vsum = 0;
        if constexpr (VLANES) {
            if (t < 24) {
                const int dir = t >> 3, v = t & 7;
                const int ib = v & 1, jb = (v >> 1) & 1, kb = v >> 2;
                const int line = dir == 0 ? jb + 2 * kb : (dir == 1 ? 4 + ib + 2 * kb : 8 + ib + 2 * jb);
                const int bit = dir == 0 ? ib : (dir == 1 ? jb : kb);
#pragma unroll
                for (int m2 = 0; m2 < NI; ++m2) {
                    const T am = ctA[m2], bm = ctB[m2];
                    vsum += (bit ? bm : am) * UE(line, m2);
                }
            }
        }
        T vsx = 0, vsy = 0, vsz = 0;
        if constexpr (VLANES) {
            vsx = __shfl(vsum, t & 7, 64);
            vsy = __shfl(vsum, (t & 7) + 8, 64);
            vsz = __shfl(vsum, (t & 7) + 16, 64);
        }
        if (vown) {
            const int q = t;
            T sx, sy, sz;
            if constexpr (VLANES) {
                sx = vsx;
                sy = vsy;
                sz = vsz;
            } else {
                T sxa = 0, sxb = 0, sya = 0, syb = 0, sza = 0, szb = 0;
#pragma unroll
                for (int m2 = 0; m2 < NI; ++m2) {
                    const T am = ctA[m2], bm = ctB[m2];
                    const T x = UE(vjb + 2 * vkb, m2), y = UE(4 + vib + 2 * vkb, m2), z = UE(8 + vib + 2 * vjb, m2);
                    sxa += am * x;
                    sxb += bm * x;
                    sya += am * y;
                    syb += bm * y;
                    sza += am * z;
                    szb += bm * z;
                }
                sx = vib ? sxb : sxa;
                sy = vjb ? syb : sya;
                sz = vkb ? szb : sza;
            }
            const T out = (d0 * m02 * m0 + (d1 + d2 + d3) * m02 * K00) * UV(q) +
                          m02 * K0p * (d1 * UV(q ^ 1) + d2 * UV(q ^ 2) + d3 * UV(q ^ 4)) +
                          m02 * (d1 * sx + d2 * sy + d3 * sz);
            uint32_t node;
            bool con;
            vertex_node(L, E, vib, vjb, vkb, &node, &con);
            if (!con && live) {
                out_store<SL, DIR && (NI > 5)>(A, vr, qr, node, (1 - vib) + 2 * (1 - vjb) + 4 * (1 - vkb), out);
                en += (double)UV(q) * (double)out;
            }
        }
        if (A.energy || en_acc) {
            if constexpr (NE > 1) {
                // sum over the element's lane group (aligned, power of two)
#pragma unroll
                for (int off = NT / 2; off > 0; off >>= 1) en += __shfl_xor(en, off, 64);
                if (t == 0 && live) A.energy[e * k + r] = en;
            } else {
                en = wave_sum(en);
                if ((t & 63) == 0) red[t >> 6] = en;
                __syncthreads();
                if (t == 0) {
                    double sum = 0.0;
                    for (int w = 0; w < NT / 64; ++w) sum += red[w];
                    if (A.energy && live) A.energy[e * k + r] = sum;
                    if (en_acc && live) en_acc[r] += sum;
                }
            }
        }
        if constexpr (!ONE) __syncthreads();  // LDS is reused by the next item
    };
    if constexpr (ONE) {
        const int64_t e = e0 + grp;
        item(e, e < n_end, r0);
    } else {
        for (int64_t i = 0; i < count; ++i) {
            const int64_t e = e0 + i * stride;
            for (uint32_t r = r0; r < r0 + nr; ++r) item(e, e < n_end, r);
        }
    }
#undef UE
#undef UV
}

// One element (all k right-hand sides); live = false runs the same code
// without any global write.
template <typename T, int NI, bool DIR>
__device__ void apply_element(const ApplyArgs<T>& A, int64_t e, ApplySmem<T, NI>& sm, double* en_acc,
                              int tid, bool live, const double* beta) {
    if constexpr (NI <= 15)
        apply_elements_cube<T, NI, DIR, false>(A, e, 1, 1, live ? e + 1 : e, 0, (uint32_t)A.k, &sm, en_acc, tid,
                                               beta);
    else
        apply_element_planes<T, NI, DIR>(A, e, sm, en_acc, tid, live, beta);
}

}  // namespace semcond
