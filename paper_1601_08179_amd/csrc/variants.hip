// The two other evaluations of the condensed operator that Sec. 7 compares
// with the transformed tensor-product form (TPT):
//
//  * TPC: Algorithm 3 in the physical (nodal GLL) basis with the tensor-product
//    suboperators of Table 1.  Per element the primary part H_BB u_B is
//    evaluated line by line from the 1D matrices (K along the lines that lie
//    in the boundary, the two end values along lines through the interior),
//    and the condensed part as u^ = sum_f H_Ef u_f (the face values mapped by
//    S^-1 (x) S^-1 = S^T M_II (x) S^T M_II, then the rank-one expansion by
//    a = S^T K_I0, b = S^T K_Ip along the normal), v^ = D^-1 u^, and
//    v_f -= H_fE v^ (line sums by a, b, then M_II S (x) M_II S).  The
//    eigenspace is processed one k-plane at a time.
//  * MMC: Algorithm 2 with the primary part included, i.e. one dense matrix
//    per element class (the element's Schur complement on all its boundary
//    nodes) applied to all elements of the class by one DGEMM; the gather R^T
//    and scatter R around it are index arithmetic on the skeleton layout.
//
// Both work on FP64 skeleton vectors in the physical basis.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"
#include "layout.h"

namespace semcond {

namespace {

// Entity id (0..25, element_entity's numbering) and node offset of local
// boundary slot s of an element: faces (n_I^2 each, w e s n b t), edges (n_I
// each, X(jb,kb), Y(ib,kb), Z(ib,jb)), vertices.  This is also the slot order
// of a one-element skeleton layout.
__device__ inline void slot_entity(int s, int NI, int* id, int* loc) {
    const int NI2 = NI * NI, NFACE = 6 * NI2, NEDGE = 12 * NI;
    if (s < NFACE) {
        *id = s / NI2;
        *loc = s - *id * NI2;
    } else if (s < NFACE + NEDGE) {
        const int q = (s - NFACE) / NI;
        *id = 6 + q;
        *loc = s - NFACE - q * NI;
    } else {
        *id = 18 + (s - NFACE - NEDGE);
        *loc = 0;
    }
}

// Local GLL indices (i, j, k) of boundary slot s (faces: w/e slot (k, j), s/n
// (k, i), b/t (j, i)).
__device__ inline void slot_coords(int s, int NI, int* i, int* j, int* k) {
    const int p = NI + 1, NI2 = NI * NI, NFACE = 6 * NI2, NEDGE = 12 * NI;
    if (s < NFACE) {
        const int f = s / NI2, loc = s - f * NI2, s1 = loc / NI + 1, s2 = loc % NI + 1;
        const int side = (f & 1) ? p : 0;
        if (f < 2) {
            *i = side; *j = s2; *k = s1;
        } else if (f < 4) {
            *i = s2; *j = side; *k = s1;
        } else {
            *i = s2; *j = s1; *k = side;
        }
    } else if (s < NFACE + NEDGE) {
        const int q = (s - NFACE) / NI, m = (s - NFACE) % NI + 1;
        const int b0 = q & 1, b1 = (q >> 1) & 1;
        if (q < 4) {
            *i = m; *j = b0 * p; *k = b1 * p;
        } else if (q < 8) {
            *i = b0 * p; *j = m; *k = b1 * p;
        } else {
            *i = b0 * p; *j = b1 * p; *k = m;
        }
    } else {
        const int q = s - NFACE - NEDGE;
        *i = (q & 1) * p; *j = ((q >> 1) & 1) * p; *k = (q >> 2) * p;
    }
}

// Boundary value at local node (i, j, k) from the gathered slots F (0 inside).
__device__ inline double bval(const double* F, int NI, int i, int j, int k) {
    const int p = NI + 1, NI2 = NI * NI, NFACE = 6 * NI2, NEDGE = 12 * NI;
    const bool bi = i == 0 || i == p, bj = j == 0 || j == p, bk = k == 0 || k == p;
    const int nb = (int)bi + (int)bj + (int)bk;
    if (nb == 0) return 0.0;
    if (nb == 1) {
        if (bi) return F[(i == p ? 1 : 0) * NI2 + (k - 1) * NI + (j - 1)];
        if (bj) return F[(j == p ? 3 : 2) * NI2 + (k - 1) * NI + (i - 1)];
        return F[(k == p ? 5 : 4) * NI2 + (j - 1) * NI + (i - 1)];
    }
    if (nb == 2) {
        if (!bi) return F[NFACE + ((j == p) + 2 * (k == p)) * NI + (i - 1)];
        if (!bj) return F[NFACE + (4 + (i == p) + 2 * (k == p)) * NI + (j - 1)];
        return F[NFACE + (8 + (i == p) + 2 * (j == p)) * NI + (k - 1)];
    }
    return F[NFACE + NEDGE + (i == p) + 2 * (j == p) + 4 * (k == p)];
}

constexpr int kTpcThreads = 512;

}  // namespace

// ---------------------------------------------------------------------------
// TPC: one workgroup per (element, RHS).  LDS: gathered boundary values F (the
// face part is overwritten by the transformed faces and then by the eigenspace
// line sums), output rows O, one eigenspace plane P and a face temporary Q,
// and the 1D tables K, S^-1, a, b, Lambda, w.
// ---------------------------------------------------------------------------

size_t tpc_smem_bytes(int p) {
    const size_t NI = p - 1, n = p + 1, NI2 = NI * NI, nslot = 6 * NI2 + 12 * NI + 8;
    return (2 * nslot + 2 * NI2 + n * n + NI2 + 3 * NI + n) * sizeof(double);
}

__global__ __launch_bounds__(kTpcThreads) void k_apply_tpc(Geo g, DevTab<double> tab, const double* __restrict__ K,
                                                           const double* __restrict__ u, double* __restrict__ v,
                                                           uint32_t ns, int64_t rs) {
    extern __shared__ double sh[];
    __shared__ int64_t ebase[26];
    __shared__ int econ[26];
    const Layout& L = g.L;
    const int p = L.p, n = p + 1, NI = L.NI, NI2 = NI * NI;
    const int NFACE = 6 * NI2, NEDGE = 12 * NI, NSLOT = NFACE + NEDGE + 8;
    double* F = sh;
    double* O = F + NSLOT;
    double* P = O + NSLOT;
    double* Q = P + NI2;
    double* Kl = Q + NI2;
    double* A = Kl + n * n;  // S^-1 = S^T M_II, row-major
    double* ta = A + NI2;
    double* tb = ta + NI;
    double* tl = tb + NI;
    double* w = tl + NI;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int64_t e = blockIdx.x;
    const int r = blockIdx.y;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    for (int t = tid; t < n * n; t += NT) Kl[t] = K[t];
    for (int t = tid; t < NI2; t += NT) A[t] = tab.Sinv[t];
    for (int t = tid; t < NI; t += NT) {
        ta[t] = tab.a[t];
        tb[t] = tab.b[t];
        tl[t] = tab.lam[t];
    }
    for (int t = tid; t < n; t += NT) w[t] = tab.w[t];
    if (tid < 26) {
        int64_t b;
        bool c;
        element_entity(L, e1, e2, e3, tid, &b, &c);
        ebase[tid] = b;
        econ[tid] = c ? 1 : 0;
    }
    __syncthreads();
    // ---- gather R^T (constrained entities read as 0)
    for (int s = tid; s < NSLOT; s += NT) {
        int id, loc;
        slot_entity(s, NI, &id, &loc);
        F[s] = econ[id] ? 0.0 : u[(ebase[id] + loc) * ns + r * rs];
    }
    __syncthreads();
    // ---- primary part: (H_e [u_B; 0])_B, line by line
    for (int s = tid; s < NSLOT; s += NT) {
        int i, j, k;
        slot_coords(s, NI, &i, &j, &k);
        const bool ii = i > 0 && i < p, ij = j > 0 && j < p, ik = k > 0 && k < p;
        double si = 0.0, sj = 0.0, sk = 0.0;
        if (ij && ik) {
            si = Kl[i * n] * bval(F, NI, 0, j, k) + Kl[i * n + p] * bval(F, NI, p, j, k);
        } else {
            for (int m = 0; m < n; ++m) si += Kl[i * n + m] * bval(F, NI, m, j, k);
        }
        if (ii && ik) {
            sj = Kl[j * n] * bval(F, NI, i, 0, k) + Kl[j * n + p] * bval(F, NI, i, p, k);
        } else {
            for (int m = 0; m < n; ++m) sj += Kl[j * n + m] * bval(F, NI, i, m, k);
        }
        if (ii && ij) {
            sk = Kl[k * n] * bval(F, NI, i, j, 0) + Kl[k * n + p] * bval(F, NI, i, j, p);
        } else {
            for (int m = 0; m < n; ++m) sk += Kl[k * n + m] * bval(F, NI, i, j, m);
        }
        O[s] = d[0] * w[i] * w[j] * w[k] * F[s] + d[1] * w[j] * w[k] * si + d[2] * w[i] * w[k] * sj +
               d[3] * w[i] * w[j] * sk;
    }
    __syncthreads();
    // ---- condensed part.  Faces to the transformed face basis in place:
    // T_f = S^-1 X_f S^-T (both face directions)
    for (int f = 0; f < 6; ++f) {
        double* X = F + f * NI2;
        for (int q = tid; q < NI2; q += NT) {
            const int s1 = q / NI, c = q % NI;
            double acc = 0.0;
            for (int m = 0; m < NI; ++m) acc += X[s1 * NI + m] * A[c * NI + m];
            Q[q] = acc;
        }
        __syncthreads();
        for (int q = tid; q < NI2; q += NT) {
            const int c1 = q / NI, c = q % NI;
            double acc = 0.0;
            for (int m = 0; m < NI; ++m) acc += A[c1 * NI + m] * Q[m * NI + c];
            X[q] = acc;
        }
        __syncthreads();
    }
    // eigenspace, one k-plane at a time: u^ = sum_f H_Ef T_f, v^ = D^-1 u^; the
    // w/e and s/n line sums of the plane replace the consumed face rows, the
    // b/t sums along k accumulate in registers (at most 2 points per thread)
    double* Tw = F;
    double* Te = F + NI2;
    double* Ts = F + 2 * NI2;
    double* Tn = F + 3 * NI2;
    double* Tb = F + 4 * NI2;
    double* Tt = F + 5 * NI2;
    double accb[2] = {0.0, 0.0}, acct[2] = {0.0, 0.0};
    for (int kk = 0; kk < NI; ++kk) {
        for (int m = 0, q = tid; q < NI2; ++m, q += NT) {
            const int j = q / NI, i = q % NI;
            const double uc = d[1] * (ta[i] * Tw[kk * NI + j] + tb[i] * Te[kk * NI + j]) +
                              d[2] * (ta[j] * Ts[kk * NI + i] + tb[j] * Tn[kk * NI + i]) +
                              d[3] * (ta[kk] * Tb[q] + tb[kk] * Tt[q]);
            const double vv = uc / (d[0] + d[1] * tl[i] + d[2] * tl[j] + d[3] * tl[kk]);
            P[q] = vv;
            accb[m] += ta[kk] * vv;
            acct[m] += tb[kk] * vv;
        }
        __syncthreads();
        for (int t = tid; t < 4 * NI; t += NT) {
            const int which = t / NI, x = t % NI;
            const double* c = (which & 1) ? tb : ta;
            double acc = 0.0;
            if (which < 2) {
                for (int m = 0; m < NI; ++m) acc += c[m] * P[x * NI + m];  // along i at (kk, j = x)
                (which ? Te : Tw)[kk * NI + x] = acc;
            } else {
                for (int m = 0; m < NI; ++m) acc += c[m] * P[m * NI + x];  // along j at (kk, i = x)
                (which == 3 ? Tn : Ts)[kk * NI + x] = acc;
            }
        }
        __syncthreads();
    }
    for (int m = 0, q = tid; q < NI2; ++m, q += NT) {
        Tb[q] = accb[m];
        Tt[q] = acct[m];
    }
    __syncthreads();
    // back to the faces: O_f -= d_f S^-T Sum_f S^-1 (M_II S (x) M_II S)
    for (int f = 0; f < 6; ++f) {
        double* X = F + f * NI2;
        const double df = f < 2 ? d[1] : (f < 4 ? d[2] : d[3]);
        for (int q = tid; q < NI2; q += NT) {
            const int s1 = q / NI, c = q % NI;
            double acc = 0.0;
            for (int m = 0; m < NI; ++m) acc += X[s1 * NI + m] * A[m * NI + c];
            Q[q] = acc;
        }
        __syncthreads();
        for (int q = tid; q < NI2; q += NT) {
            const int c1 = q / NI, c = q % NI;
            double acc = 0.0;
            for (int m = 0; m < NI; ++m) acc += A[m * NI + c1] * Q[m * NI + c];
            O[f * NI2 + q] -= df * acc;
        }
        __syncthreads();
    }
    // ---- scatter R
    for (int s = tid; s < NSLOT; s += NT) {
        int id, loc;
        slot_entity(s, NI, &id, &loc);
        if (!econ[id]) atomic_add(&v[(ebase[id] + loc) * ns + r * rs], O[s]);
    }
}

hipError_t launch_apply_tpc(const Geo& g, const DevTab<double>& tab, const double* K, const double* u, double* v,
                            int k, hipStream_t st) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    if (ne <= 0) return hipSuccess;
    if (ne > INT32_MAX) return hipErrorInvalidValue;
    const size_t shm = tpc_smem_bytes(g.L.p);
    hipLaunchKernelGGL(k_apply_tpc, dim3((unsigned)ne, (unsigned)k), dim3(kTpcThreads), shm, st, g, tab, K, u, v,
                       (uint32_t)k, (int64_t)1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MMC: the element metrics (for grouping elements into classes), and the
// gather / scatter around the class GEMMs.  UL and VL are column-major
// (n_B x n_cols): column col_of[e] * k + r holds element e's boundary values of
// RHS r in local slot order.
// ---------------------------------------------------------------------------

__global__ void k_elem_metrics(Geo g, double* __restrict__ d) {
    const Layout& L = g.L;
    const int64_t ne = (int64_t)L.n1 * L.n2 * L.n3;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        int e1, e2, e3;
        elem_index(L, e, &e1, &e2, &e3);
        double dd[4];
        elem_metric(g, e, e1, e2, e3, dd);
        for (int m = 0; m < 4; ++m) d[4 * e + m] = dd[m];
    }
}

hipError_t launch_elem_metrics(const Geo& g, double* d, hipStream_t st) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    int64_t b = (ne + 255) / 256;
    if (b > 65536) b = 65536;
    if (b > 0) hipLaunchKernelGGL(k_elem_metrics, dim3((unsigned)b), dim3(256), 0, st, g, d);
    return hipGetLastError();
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_mmc_move(Layout L, const int* __restrict__ col_of, int k,
                                                  const double* __restrict__ u, double* __restrict__ v,
                                                  double* __restrict__ UL, const double* __restrict__ VL) {
    __shared__ int64_t ebase[26];
    __shared__ int econ[26];
    const int NI = L.NI, NSLOT = 6 * NI * NI + 12 * NI + 8;
    const int64_t e = blockIdx.x;
    const int r = blockIdx.y;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    if (threadIdx.x < 26) {
        int64_t b;
        bool c;
        element_entity(L, e1, e2, e3, threadIdx.x, &b, &c);
        ebase[threadIdx.x] = b;
        econ[threadIdx.x] = c ? 1 : 0;
    }
    __syncthreads();
    const int64_t col = (int64_t)col_of[e] * k + r;
    for (int s = threadIdx.x; s < NSLOT; s += blockDim.x) {
        int id, loc;
        slot_entity(s, NI, &id, &loc);
        const int64_t node = ebase[id] + loc;
        if (SCATTER) {
            if (!econ[id]) atomic_add(&v[node * k + r], VL[col * NSLOT + s]);
        } else {
            UL[col * NSLOT + s] = econ[id] ? 0.0 : u[node * k + r];
        }
    }
}

hipError_t launch_mmc_gather(const Layout& L, const int* col_of, const double* u, double* UL, int k, hipStream_t st) {
    const int64_t ne = (int64_t)L.n1 * L.n2 * L.n3;
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mmc_move<false>, dim3((unsigned)ne, (unsigned)k), dim3(256), 0, st, L, col_of, k, u,
                       (double*)nullptr, UL, (const double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_mmc_scatter(const Layout& L, const int* col_of, const double* VL, double* v, int k, hipStream_t st) {
    const int64_t ne = (int64_t)L.n1 * L.n2 * L.n3;
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mmc_move<true>, dim3((unsigned)ne, (unsigned)k), dim3(256), 0, st, L, col_of, k,
                       (const double*)nullptr, v, (double*)nullptr, VL);
    return hipGetLastError();
}

}  // namespace semcond
