// Basis changes, preconditioner diagonal, right-hand-side condensation,
// interior recovery, nodal/skeleton copies and the conjugate-gradient vector
// kernels of the BT solver.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "cg_device.h"
#include "device_common.h"
#include "kernels.h"
#include "rhs_lines.h"
#include "tables.h"

namespace semcond {

// ---------------------------------------------------------------------------
// Basis change of skeleton arrays (Sec. 6: T = S1(x)S1(x)S1, S1 = diag(1,S,1),
// acts on a face through its two interior axes and on an edge through one).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(1024) void k_transform_faces(Layout L, const T* __restrict__ A,
                                                          const T* __restrict__ in, T* __restrict__ out,
                                                          int k, int fpb, int64_t nfaces, uint32_t ns, int64_t rs) {
    extern __shared__ unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NI = L.NI, NI2 = NI * NI;
    T* Y = X + fpb * NI2;
    const int t = threadIdx.x;
    const int lf = t / NI2, loc = t - lf * NI2;
    const int64_t face = (int64_t)blockIdx.x * fpb + lf;
    const bool valid = lf < fpb && face < nfaces;
    const int s1 = loc / NI, s2 = loc - (loc / NI) * NI;
    const int64_t node = face * NI2 + loc;  // faces are contiguous from oFx = 0
    for (int r = 0; r < k; ++r) {
        if (valid) X[t] = in[node * ns + r * rs];
        __syncthreads();
        if (valid) {  // along the fast axis: Y(s1, c) = sum_c' A[c][c'] X(s1, c')
            T acc = 0;
            for (int m = 0; m < NI; ++m) acc += A[s2 * NI + m] * X[lf * NI2 + s1 * NI + m];
            Y[t] = acc;
        }
        __syncthreads();
        if (valid) {  // along the slow axis
            T acc = 0;
            for (int m = 0; m < NI; ++m) acc += A[s1 * NI + m] * Y[lf * NI2 + m * NI + s2];
            out[node * ns + r * rs] = acc;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void k_transform_edges(Layout L, const T* __restrict__ A, const T* __restrict__ in,
                                  T* __restrict__ out, int k, uint32_t ns, int64_t rs) {
    const int64_t nval = (L.Ns - L.oEx) * k;
    const int NI = L.NI;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nval;
         idx += (int64_t)gridDim.x * blockDim.x) {
        // consecutive threads on consecutive entries of the layout
        const int64_t nv = L.Ns - L.oEx;
        const bool nm = rs == 1;
        const int64_t s = L.oEx + (nm ? idx / k : idx % nv);
        const int r = (int)(nm ? idx % k : idx / nv);
        if (s >= L.oV) {
            out[s * ns + r * rs] = in[s * ns + r * rs];
        } else {
            const int64_t t = s - L.oEx;
            const int64_t base = L.oEx + (t / NI) * NI;
            const int m = (int)(t % NI);
            T acc = 0;
            for (int m2 = 0; m2 < NI; ++m2) acc += A[m * NI + m2] * in[(base + m2) * ns + r * rs];
            out[s * ns + r * rs] = acc;
        }
    }
}

template <typename T>
hipError_t launch_transform(const Layout& L, const T* A, const T* in, T* out, int k, hipStream_t st,
                            SkelStride sk) {
    sk = skel_stride(sk, k);
    const int NI2 = L.NI * L.NI;
    const int64_t nfaces = L.oEx / NI2;
    int fpb = 1024 / NI2;
    if (fpb < 1) fpb = 1;
    if (fpb > 64) fpb = 64;
    int threads = ((fpb * NI2 + 63) / 64) * 64;
    int64_t blocks = (nfaces + fpb - 1) / fpb;
    size_t shm = 2 * (size_t)fpb * NI2 * sizeof(T);
    if (blocks > 0)
        hipLaunchKernelGGL(k_transform_faces<T>, dim3((unsigned)blocks), dim3(threads), shm, st, L, A, in,
                           out, k, fpb, nfaces, sk.ns, sk.rs);
    int64_t nval = (L.Ns - L.oEx) * k;
    int eb = (int)((nval + 255) / 256);
    if (eb > 65536) eb = 65536;
    if (eb > 0) hipLaunchKernelGGL(k_transform_edges<T>, dim3(eb), dim3(256), 0, st, L, A, in, out, k, sk.ns, sk.rs);
    return hipGetLastError();
}

template hipError_t launch_transform<double>(const Layout&, const double*, const double*, double*, int,
                                             hipStream_t, SkelStride);
template hipError_t launch_transform<float>(const Layout&, const float*, const float*, float*, int,
                                            hipStream_t, SkelStride);

// ---------------------------------------------------------------------------
// Assembly R from per-side slots (layout.h): out(node, r) = the node's slots of
// right-hand side r summed in slot order, written at node * ns + r * rs.
// Slots that no element wrote hold 0, so constrained nodes receive 0.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_slot_sum(Layout L, const T* __restrict__ qs, int64_t qlen, T* __restrict__ out, int k, uint32_t ns,
                           uint32_t rs) {
    const int64_t n_all = L.Ns * k;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_all; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / L.Ns);
        const uint32_t node = (uint32_t)(i - (int64_t)r * L.Ns);
        out[(int64_t)node * ns + (int64_t)r * rs] = slot_sum(L, qs + (int64_t)r * qlen, node);
    }
}

template <typename T>
hipError_t launch_slot_sum(const Layout& L, const T* slots, int64_t qlen, T* out, int k, uint32_t ns, uint32_t rs,
                           hipStream_t st) {
    int64_t b = (L.Ns * k + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) return hipSuccess;
    hipLaunchKernelGGL(k_slot_sum<T>, dim3((unsigned)b), dim3(256), 0, st, L, slots, qlen, out, k, ns, rs);
    return hipGetLastError();
}
template hipError_t launch_slot_sum<double>(const Layout&, const double*, int64_t, double*, int, uint32_t, uint32_t,
                                            hipStream_t);
template hipError_t launch_slot_sum<float>(const Layout&, const float*, int64_t, float*, int, uint32_t, uint32_t,
                                           hipStream_t);

// ---------------------------------------------------------------------------
// Preconditioner: diagonal of the transformed condensed operator (Sec. 8: the
// block preconditioner is diagonal in the transformed system).  Per element:
//   face w (k,j): d0 M00 + d1 K00 + d2 M00 L_j + d3 M00 L_k - d1^2 sum_i a_i^2 / D_kji
//   (e: b_i; s/n and b/t analogous along j and k)
//   edge along x1 (i): d0 M00^2 + d1 M00^2 L_i + (d2+d3) M00 K00 (others analogous)
//   vertex: d0 M00^3 + (d1+d2+d3) M00^2 K00
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_precond_diag(Geo g, DevTab<double> tab, double* __restrict__ diag,
                                                      double* __restrict__ slots) {
    const Layout& L = g.L;
    const int NI = L.NI, NI2 = NI * NI;
    const int64_t e = blockIdx.x;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    const double m0 = tab.m0, K00 = tab.K00;
    const int nslot = 6 * NI2 + 12 * NI + 8;
    for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
        int ent, loc;
        double val;
        if (s < 6 * NI2) {
            const int f = s / NI2;
            loc = s - f * NI2;
            ent = f;
            const int s1 = loc / NI, s2 = loc % NI;
            const double* c = (f & 1) ? tab.b : tab.a;
            double cond = 0.0;
            if (f < 2) {  // (k, j), line along i
                for (int m = 0; m < NI; ++m)
                    cond += c[m] * c[m] / (d[0] + d[1] * tab.lam[m] + d[2] * tab.lam[s2] + d[3] * tab.lam[s1]);
                val = d[0] * m0 + d[1] * K00 + d[2] * m0 * tab.lam[s2] + d[3] * m0 * tab.lam[s1] - d[1] * d[1] * cond;
            } else if (f < 4) {  // (k, i), line along j
                for (int m = 0; m < NI; ++m)
                    cond += c[m] * c[m] / (d[0] + d[1] * tab.lam[s2] + d[2] * tab.lam[m] + d[3] * tab.lam[s1]);
                val = d[0] * m0 + d[2] * K00 + d[1] * m0 * tab.lam[s2] + d[3] * m0 * tab.lam[s1] - d[2] * d[2] * cond;
            } else {  // (j, i), line along k
                for (int m = 0; m < NI; ++m)
                    cond += c[m] * c[m] / (d[0] + d[1] * tab.lam[s2] + d[2] * tab.lam[s1] + d[3] * tab.lam[m]);
                val = d[0] * m0 + d[3] * K00 + d[1] * m0 * tab.lam[s2] + d[2] * m0 * tab.lam[s1] - d[3] * d[3] * cond;
            }
        } else if (s < 6 * NI2 + 12 * NI) {
            const int q = (s - 6 * NI2) / NI;
            loc = s - 6 * NI2 - q * NI;
            ent = 6 + q;
            const double l = tab.lam[loc];
            if (q < 4)
                val = d[0] * m0 * m0 + d[1] * m0 * m0 * l + (d[2] + d[3]) * m0 * K00;
            else if (q < 8)
                val = d[0] * m0 * m0 + d[2] * m0 * m0 * l + (d[1] + d[3]) * m0 * K00;
            else
                val = d[0] * m0 * m0 + d[3] * m0 * m0 * l + (d[1] + d[2]) * m0 * K00;
        } else {
            ent = 18 + (s - 6 * NI2 - 12 * NI);
            loc = 0;
            val = d[0] * m0 * m0 * m0 + (d[1] + d[2] + d[3]) * m0 * m0 * K00;
        }
        int64_t base;
        bool con;
        element_entity(L, e1, e2, e3, ent, &base, &con);
        if (con) continue;
        if (slots)
            slots[slot_addr(L, (uint32_t)(base + loc), entity_slot(ent))] = val;
        else
            atomic_add(&diag[base + loc], val);
    }
}

hipError_t launch_precond_diag(const Geo& g, const DevTab<double>& tab, double* diag, double* slots,
                               hipStream_t st) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    hipLaunchKernelGGL(k_precond_diag, dim3((unsigned)ne), dim3(256), 0, st, g, tab, diag, slots);
    if (slots) return launch_slot_sum<double>(g.L, slots, slot_len(g.L), diag, 1, 1, 1, st);
    return hipGetLastError();
}

template <typename T>
__global__ void k_precond_invert(Layout L, const double* __restrict__ diag, T* __restrict__ pinv) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < L.Ns;
         s += (int64_t)gridDim.x * blockDim.x) {
        int I1, I2, I3;
        bool con;
        skeleton_node(L, s, &I1, &I2, &I3, &con);
        pinv[s] = con ? (T)0 : (T)(1.0 / diag[s]);
    }
}

template <typename T>
hipError_t launch_precond_invert(const Layout& L, const double* diag, T* pinv, hipStream_t st) {
    int blocks = (int)((L.Ns + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_precond_invert<T>, dim3(blocks), dim3(256), 0, st, L, diag, pinv);
    return hipGetLastError();
}
template hipError_t launch_precond_invert<double>(const Layout&, const double*, double*, hipStream_t);
template hipError_t launch_precond_invert<float>(const Layout&, const double*, float*, hipStream_t);

// D of the fast diagonalisation (eq. hii_diagonal) at every interior point of
// one metric class, inverted with a correctly rounded FP64 division and
// rounded to FP32.
__global__ void k_dinv_table(const double* __restrict__ lam, int NI, const double* __restrict__ dclass, int nc,
                             float* __restrict__ out) {
    const int64_t n3 = (int64_t)NI * NI * NI, total = n3 * nc;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = x / n3, r = x - c * n3;
        const int kk = (int)(r / (NI * NI)), j = (int)((r / NI) % NI), i = (int)(r % NI);
        const double* d = dclass + 4 * c;
        const double D = __builtin_fma(d[3], lam[kk], __builtin_fma(d[2], lam[j], __builtin_fma(d[1], lam[i], d[0])));
        out[x] = (float)(1.0 / D);
    }
}

hipError_t launch_dinv_table(const double* lam, int NI, const double* dclass, int nc, float* out, hipStream_t st) {
    const int64_t total = (int64_t)NI * NI * NI * nc;
    int64_t b = (total + 255) / 256;
    if (b > 65536) b = 65536;
    if (b > 0) hipLaunchKernelGGL(k_dinv_table, dim3((unsigned)b), dim3(256), 0, st, lam, NI, dclass, nc, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Element cube helpers: 1D transforms along the lines of a (p+1)^3 cube,
// acting on the interior indices 1..n_I of each line.
// ---------------------------------------------------------------------------

// axis 0: lines along i (fixed kk, jj); 1: along j; 2: along k.
// interior_only: restrict to lines whose two fixed indices are interior.
__device__ void cube_lines(double* cube, int p, int axis, const double* __restrict__ A, bool interior_only) {
    const int n = p + 1, NI = p - 1;
    const int nl = interior_only ? NI * NI : n * n;
    const int stride = axis == 0 ? 1 : (axis == 1 ? n : n * n);
    for (int l = threadIdx.x; l < nl; l += blockDim.x) {
        int u = l / (interior_only ? NI : n), w = l % (interior_only ? NI : n);
        if (interior_only) { u += 1; w += 1; }
        // (u, w) are the two fixed indices in (slow, fast) order of the remaining axes
        int base;
        if (axis == 0) base = (u * n + w) * n;       // (kk, jj)
        else if (axis == 1) base = u * n * n + w;     // (kk, ii)
        else base = u * n + w;                        // (jj, ii)
        double x[kMaxNI];
#pragma unroll
        for (int m = 0; m < kMaxNI; ++m)
            if (m < NI) x[m] = cube[base + (1 + m) * stride];
        for (int m = 0; m < NI; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int m2 = 0; m2 < kMaxNI; ++m2)
                if (m2 < NI) acc += A[m * NI + m2] * x[m2];
            cube[base + (1 + m) * stride] = acc;
        }
    }
}

// cube(kk,jj,ii) = J w_ii w_jj w_kk f(node) then F~ = (S1^T (x) S1^T (x) S1^T) F.
__device__ void cube_transformed_rhs(double* cube, const Geo& g, const DevTab<double>& tab,
                                     const double* __restrict__ St, const double* __restrict__ f, int64_t N,
                                     int r, int e1, int e2, int e3) {
    const Layout& L = g.L;
    const int p = L.p, n = p + 1;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    const double J = elem_jacobian(g, e1, e2, e3);
    for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
        const int ii = idx % n, jj = (idx / n) % n, kk = idx / (n * n);
        const int64_t node = ((int64_t)e1 * p + ii) + N1 * (((int64_t)e2 * p + jj) + N2 * ((int64_t)e3 * p + kk));
        cube[idx] = J * tab.w[ii] * tab.w[jj] * tab.w[kk] * f[(int64_t)r * N + node];
    }
    __syncthreads();
    cube_lines(cube, p, 0, St, false);
    __syncthreads();
    cube_lines(cube, p, 1, St, false);
    __syncthreads();
    cube_lines(cube, p, 2, St, false);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Condensed transformed right-hand side (Algorithm 4, first loop):
//   F^~_f = F~_f - H~_FI D^-1 F~_I on the six faces, F~ on edges and vertices.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_condense_rhs(Geo g, DevTab<double> tab, const double* __restrict__ f,
                                                      int64_t N, double* __restrict__ fhat, int k, double* scratch,
                                                      double* __restrict__ slots, int64_t qlen, uint32_t ns,
                                                      int64_t rs) {
    extern __shared__ double cube_lds[];
    const Layout& L = g.L;
    const int p = L.p, n = p + 1, NI = L.NI, NI2 = NI * NI;
    const int64_t ne = (int64_t)L.n1 * L.n2 * L.n3;
    double* cube = scratch ? scratch + (int64_t)blockIdx.x * n * n * n : cube_lds;
    const int nslot = 6 * NI2 + 12 * NI + 8;
#define C(kk, jj, ii) cube[((kk) * n + (jj)) * n + (ii)]
    for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
        int e1, e2, e3;
        elem_index(L, e, &e1, &e2, &e3);
        double d[4];
        elem_metric(g, e, e1, e2, e3, d);
        for (int r = 0; r < k; ++r) {
            cube_transformed_rhs(cube, g, tab, tab.St, f, N, r, e1, e2, e3);
            for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
                int ent, loc;
                double val;
                if (s < 6 * NI2) {
                    const int fc = s / NI2;
                    loc = s - fc * NI2;
                    ent = fc;
                    const int s1 = loc / NI, s2 = loc % NI;
                    const double* c = (fc & 1) ? tab.b : tab.a;
                    const int side = (fc & 1) ? p : 0;
                    double acc = 0.0;
                    if (fc < 2) {  // (k, j), sum over i
                        for (int m = 0; m < NI; ++m)
                            acc += c[m] * C(1 + s1, 1 + s2, 1 + m) /
                                   (d[0] + d[1] * tab.lam[m] + d[2] * tab.lam[s2] + d[3] * tab.lam[s1]);
                        val = C(1 + s1, 1 + s2, side) - d[1] * acc;
                    } else if (fc < 4) {  // (k, i), sum over j
                        for (int m = 0; m < NI; ++m)
                            acc += c[m] * C(1 + s1, 1 + m, 1 + s2) /
                                   (d[0] + d[1] * tab.lam[s2] + d[2] * tab.lam[m] + d[3] * tab.lam[s1]);
                        val = C(1 + s1, side, 1 + s2) - d[2] * acc;
                    } else {  // (j, i), sum over k
                        for (int m = 0; m < NI; ++m)
                            acc += c[m] * C(1 + m, 1 + s1, 1 + s2) /
                                   (d[0] + d[1] * tab.lam[s2] + d[2] * tab.lam[s1] + d[3] * tab.lam[m]);
                        val = C(side, 1 + s1, 1 + s2) - d[3] * acc;
                    }
                } else if (s < 6 * NI2 + 12 * NI) {
                    const int q = (s - 6 * NI2) / NI;
                    loc = s - 6 * NI2 - q * NI;
                    ent = 6 + q;
                    if (q < 4) {
                        const int jb = q & 1, kb = q >> 1;
                        val = C(kb * p, jb * p, 1 + loc);
                    } else if (q < 8) {
                        const int ib = (q - 4) & 1, kb = (q - 4) >> 1;
                        val = C(kb * p, 1 + loc, ib * p);
                    } else {
                        const int ib = (q - 8) & 1, jb = (q - 8) >> 1;
                        val = C(1 + loc, jb * p, ib * p);
                    }
                } else {
                    const int q = s - 6 * NI2 - 12 * NI;
                    ent = 18 + q;
                    loc = 0;
                    val = C((q >> 2) * p, ((q >> 1) & 1) * p, (q & 1) * p);
                }
                int64_t base;
                bool con;
                element_entity(L, e1, e2, e3, ent, &base, &con);
                if (con) continue;
                if (slots)
                    slots[(int64_t)r * qlen + slot_addr(L, (uint32_t)(base + loc), entity_slot(ent))] = val;
                else
                    atomic_add(&fhat[(base + loc) * ns + r * rs], val);
            }
            __syncthreads();
        }
    }
#undef C
}

// Element-cube pieces (RhsSmem, line transforms): rhs_lines.h.

// C(kk,jj,ii) = J w_ii w_jj w_kk f(node) of RHS r, then (S1 (x) S1 (x) S1)-type
// transform by sm.A along the three axes (all lines).
template <int NI>
__device__ void rhs_cube(RhsSmem<NI>& sm, const Geo& g, const double* __restrict__ f, int64_t N, int r, int e1,
                         int e2, int e3, double J) {
    constexpr int n = NI + 2, p = NI + 1;
    const Layout& L = g.L;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
        const int ii = idx % n, jj = (idx / n) % n, kk = idx / (n * n);
        const int64_t node = ((int64_t)e1 * p + ii) + N1 * (((int64_t)e2 * p + jj) + N2 * ((int64_t)e3 * p + kk));
        sm.C[idx] = J * sm.w[ii] * sm.w[jj] * sm.w[kk] * f[(int64_t)r * N + node];
    }
    __syncthreads();
    if constexpr (rhs_mfma<NI>()) {
        LineMat<NI> B;
        line_mat<NI>(B, sm.A);
        rhs_lines_mfma<NI, 0>(sm.C, B, 0);
        __syncthreads();
        rhs_lines_mfma<NI, 1>(sm.C, B, 0);
        __syncthreads();
        rhs_lines_mfma<NI, 2>(sm.C, B, 0);
        __syncthreads();
    } else {
        rhs_lines<NI, 0>(sm.C, sm.A, 0);
        __syncthreads();
        rhs_lines<NI, 1>(sm.C, sm.A, 0);
        __syncthreads();
        rhs_lines<NI, 2>(sm.C, sm.A, 0);
        __syncthreads();
    }
}

template <int NI>
__global__ __launch_bounds__(kRhsThreads) void k_condense_rhs_t(Geo g, DevTab<double> tab,
                                                                const double* __restrict__ f, int64_t N,
                                                                double* __restrict__ fhat, int k,
                                                                double* __restrict__ slots, int64_t qlen,
                                                                uint32_t ns, int64_t rs) {
    constexpr int n = NI + 2, p = NI + 1, NI2 = NI * NI;
    constexpr int nslot = 6 * NI2 + 12 * NI + 8;
    __shared__ RhsSmem<NI> sm;
    const Layout& L = g.L;
    const int64_t e = blockIdx.x;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    const double J = elem_jacobian(g, e1, e2, e3);
    rhs_tables<NI>(sm, tab, tab.St);
#define C(kk, jj, ii) sm.C[((kk) * n + (jj)) * n + (ii)]
    {
        const int r = blockIdx.y;  // one workgroup per (element, right-hand side)
        __syncthreads();  // tables stored
        rhs_cube<NI>(sm, g, f, N, r, e1, e2, e3, J);
        // interior: V = D^-1 F~_I
        for (int idx = threadIdx.x; idx < NI2 * NI; idx += blockDim.x) {
            const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
            C(1 + kk, 1 + j, 1 + i) *= recip<double>(d[0] + d[1] * sm.lam[i] + d[2] * sm.lam[j] + d[3] * sm.lam[kk]);
        }
        __syncthreads();
        for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
            int ent, loc;
            const double val = condensed_row<NI>(sm, s, d, &ent, &loc);
            int64_t base;
            bool con;
            element_entity(L, e1, e2, e3, ent, &base, &con);
            if (con) continue;
            if (slots)
                slots[(int64_t)r * qlen + slot_addr(L, (uint32_t)(base + loc), entity_slot(ent))] = val;
            else
                atomic_add(&fhat[(base + loc) * ns + r * rs], val);
        }
    }
#undef C
}

template <int NI>
__global__ __launch_bounds__(kRhsThreads) void k_recover_interior_t(Geo g, DevTab<double> tab,
                                                                    const double* __restrict__ f, int64_t N,
                                                                    const double* __restrict__ xs,
                                                                    double* __restrict__ u, int k, int keep_con,
                                                                    uint32_t ns, int64_t rs) {
    constexpr int n = NI + 2, p = NI + 1, NI2 = NI * NI;
    __shared__ RhsSmem<NI> sm;
    __shared__ int64_t fb[6];
    __shared__ int fcon[6];
    const Layout& L = g.L;
    const int64_t e = blockIdx.x;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    double d[4];
    elem_metric(g, e, e1, e2, e3, d);
    const double J = elem_jacobian(g, e1, e2, e3);
    if (threadIdx.x < 6) {
        bool c;
        element_entity(L, e1, e2, e3, threadIdx.x, &fb[threadIdx.x], &c);
        fcon[threadIdx.x] = c && !keep_con ? 1 : 0;
    }
    // forward transform by S^T first; S for the back transform afterwards
#define C(kk, jj, ii) sm.C[((kk) * n + (jj)) * n + (ii)]
#define UF(face, s1, s2) (fcon[face] ? 0.0 : xs[(fb[face] + (int64_t)(s1) * NI + (s2)) * ns + r * rs])
    {
        const int r = blockIdx.y;  // one workgroup per (element, right-hand side)
        __syncthreads();  // face bases and flags stored
        rhs_tables<NI>(sm, tab, tab.St);
        __syncthreads();
        rhs_cube<NI>(sm, g, f, N, r, e1, e2, e3, J);
        for (int idx = threadIdx.x; idx < NI2 * NI; idx += blockDim.x) {
            const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
            const double uc = d[1] * (sm.a[i] * UF(0, kk, j) + sm.b[i] * UF(1, kk, j)) +
                              d[2] * (sm.a[j] * UF(2, kk, i) + sm.b[j] * UF(3, kk, i)) +
                              d[3] * (sm.a[kk] * UF(4, j, i) + sm.b[kk] * UF(5, j, i));
            const double D = d[0] + d[1] * sm.lam[i] + d[2] * sm.lam[j] + d[3] * sm.lam[kk];
            C(1 + kk, 1 + j, 1 + i) = (C(1 + kk, 1 + j, 1 + i) - uc) * recip<double>(D);
        }
        for (int t = threadIdx.x; t < NI * NI; t += blockDim.x) sm.A[t] = tab.S[t];  // read only after the barrier
        __syncthreads();
        if constexpr (rhs_mfma<NI>()) {
            LineMat<NI> B;
            line_mat<NI>(B, sm.A);
            rhs_lines_mfma<NI, 0>(sm.C, B, 1);
            __syncthreads();
            rhs_lines_mfma<NI, 1>(sm.C, B, 1);
            __syncthreads();
            rhs_lines_mfma<NI, 2>(sm.C, B, 1);
            __syncthreads();
        } else {
            rhs_lines<NI, 0>(sm.C, sm.A, 1);
            __syncthreads();
            rhs_lines<NI, 1>(sm.C, sm.A, 1);
            __syncthreads();
            rhs_lines<NI, 2>(sm.C, sm.A, 1);
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < NI2 * NI; idx += blockDim.x) {
            const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
            const int64_t node =
                ((int64_t)e1 * p + 1 + i) + N1 * (((int64_t)e2 * p + 1 + j) + N2 * ((int64_t)e3 * p + 1 + kk));
            u[(int64_t)r * N + node] = C(1 + kk, 1 + j, 1 + i);
        }
    }
#undef UF
#undef C
}

int rhs_grid_for_scratch(int p, int64_t n_e, bool* needs_scratch) {
    const size_t bytes = (size_t)(p + 1) * (p + 1) * (p + 1) * sizeof(double);
    *needs_scratch = bytes > 64 * 1024;
    int64_t grid = n_e;
    if (*needs_scratch && grid > 2048) grid = 2048;
    if (grid > (1 << 30)) grid = 1 << 30;
    return (int)grid;
}

#define RHS_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

hipError_t launch_condense_rhs(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                               double* fhat, int k, double* scratch, int grid, double* slots, hipStream_t st,
                               SkelStride sk, int rhs_batch) {
    sk = skel_stride(sk, k);
    const int64_t qlen = slot_len(g.L);
    hipError_t e = launch_condense_rhs_body(g, tab, f, N, fhat, k, scratch, grid, slots, qlen, st, sk, rhs_batch);
    if (e != hipSuccess || !slots) return e;
    return launch_slot_sum<double>(g.L, slots, qlen, fhat, k, sk.ns, (uint32_t)sk.rs, st);
}

hipError_t launch_condense_rhs_body(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                    double* fhat, int k, double* scratch, int grid, double* slots, int64_t qlen,
                                    hipStream_t st, SkelStride sk, int rhs_batch) {
    sk = skel_stride(sk, k);
    if (rhs_batch > 0 && rhs_batched_supported(g.L, N))
        return launch_condense_rhs_mb(g, tab, f, N, fhat, k, rhs_batch, slots, qlen, st, sk);
    if (g.L.NI <= 15) {
        const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
        if (ne <= 0) return hipSuccess;
        if (ne > INT32_MAX) return hipErrorInvalidValue;
        switch (g.L.NI) {
#define X(NI)                                                                                                    \
    case NI:                                                                                                     \
        hipLaunchKernelGGL(k_condense_rhs_t<NI>, dim3((unsigned)ne, (unsigned)k), dim3(kRhsThreads), 0, st, g, tab, \
                           f, N, fhat, k, slots, qlen, sk.ns, sk.rs);                                            \
        break;
            RHS_CASES(X)
#undef X
        }
        return hipGetLastError();
    }
    const int n = g.L.p + 1;
    const size_t shm = scratch ? 0 : (size_t)n * n * n * sizeof(double);
    hipLaunchKernelGGL(k_condense_rhs, dim3(grid), dim3(256), shm, st, g, tab, f, N, fhat, k, scratch, slots, qlen,
                       sk.ns, sk.rs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interior recovery and back-transform (Algorithm 4, second loop):
//   u~_I = D^-1 (F~_I - H~_IB u~_B),  u_I = (S(x)S(x)S) u~_I,
// with H~_IB u~_B = d1 (a_i U_w + b_i U_e) + d2 (a_j U_s + b_j U_n) + d3 (a_k U_b + b_k U_t)
// (Table 2).  Writes the interior nodes of the element into u [k][N].
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_recover_interior(Geo g, DevTab<double> tab, const double* __restrict__ f,
                                                          int64_t N, const double* __restrict__ xs,
                                                          double* __restrict__ u, int k, double* scratch,
                                                          int keep_con, uint32_t ns, int64_t rs) {
    extern __shared__ double cube_lds[];
    __shared__ int64_t fb[6];
    __shared__ int fc[6];
    const Layout& L = g.L;
    const int p = L.p, n = p + 1, NI = L.NI, NI2 = NI * NI;
    const int64_t ne = (int64_t)L.n1 * L.n2 * L.n3;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    double* cube = scratch ? scratch + (int64_t)blockIdx.x * n * n * n : cube_lds;
#define C(kk, jj, ii) cube[((kk) * n + (jj)) * n + (ii)]
    for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
        int e1, e2, e3;
        elem_index(L, e, &e1, &e2, &e3);
        double d[4];
        elem_metric(g, e, e1, e2, e3, d);
        if (threadIdx.x < 6) {
            bool c;
            element_entity(L, e1, e2, e3, threadIdx.x, &fb[threadIdx.x], &c);
            fc[threadIdx.x] = c ? 1 : 0;
        }
        for (int r = 0; r < k; ++r) {
            cube_transformed_rhs(cube, g, tab, tab.St, f, N, r, e1, e2, e3);
#define UF(face, s1, s2) ((fc[face] && !keep_con) ? 0.0 : xs[(fb[face] + (int64_t)(s1) * NI + (s2)) * ns + r * rs])
            for (int idx = threadIdx.x; idx < NI2 * NI; idx += blockDim.x) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                const double uc = d[1] * (tab.a[i] * UF(0, kk, j) + tab.b[i] * UF(1, kk, j)) +
                                  d[2] * (tab.a[j] * UF(2, kk, i) + tab.b[j] * UF(3, kk, i)) +
                                  d[3] * (tab.a[kk] * UF(4, j, i) + tab.b[kk] * UF(5, j, i));
                const double D = d[0] + d[1] * tab.lam[i] + d[2] * tab.lam[j] + d[3] * tab.lam[kk];
                C(1 + kk, 1 + j, 1 + i) = (C(1 + kk, 1 + j, 1 + i) - uc) / D;
            }
#undef UF
            __syncthreads();
            cube_lines(cube, p, 0, tab.S, true);
            __syncthreads();
            cube_lines(cube, p, 1, tab.S, true);
            __syncthreads();
            cube_lines(cube, p, 2, tab.S, true);
            __syncthreads();
            for (int idx = threadIdx.x; idx < NI2 * NI; idx += blockDim.x) {
                const int i = idx % NI, j = (idx / NI) % NI, kk = idx / NI2;
                const int64_t node = ((int64_t)e1 * p + 1 + i) +
                                     N1 * (((int64_t)e2 * p + 1 + j) + N2 * ((int64_t)e3 * p + 1 + kk));
                u[(int64_t)r * N + node] = C(1 + kk, 1 + j, 1 + i);
            }
            __syncthreads();
        }
    }
#undef C
}

hipError_t launch_recover_interior(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                   const double* xskel, double* u, int k, double* scratch, int grid,
                                   int keep_con, hipStream_t st, SkelStride sk, int rhs_batch) {
    sk = skel_stride(sk, k);
    if (rhs_batch > 0 && rhs_batched_supported(g.L, N))
        return launch_recover_interior_mb(g, tab, f, N, xskel, u, k, rhs_batch, keep_con, st, sk);
    if (g.L.NI <= 15) {
        const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
        if (ne <= 0) return hipSuccess;
        if (ne > INT32_MAX) return hipErrorInvalidValue;
        switch (g.L.NI) {
#define X(NI)                                                                                                  \
    case NI:                                                                                                   \
        hipLaunchKernelGGL(k_recover_interior_t<NI>, dim3((unsigned)ne, (unsigned)k), dim3(kRhsThreads), 0, st, g,  \
                           tab, f, N, xskel, u, k, keep_con, sk.ns, sk.rs);                                     \
        break;
            RHS_CASES(X)
#undef X
        }
        return hipGetLastError();
    }
    const int n = g.L.p + 1;
    const size_t shm = scratch ? 0 : (size_t)n * n * n * sizeof(double);
    hipLaunchKernelGGL(k_recover_interior, dim3(grid), dim3(256), shm, st, g, tab, f, N, xskel, u, k, scratch,
                       keep_con, sk.ns, sk.rs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Skeleton <-> nodal copies.
// ---------------------------------------------------------------------------

__device__ inline int64_t skel_nodal_index(const Layout& L, int64_t s, bool* con) {
    int I1, I2, I3;
    skeleton_node(L, s, &I1, &I2, &I3, con);
    const int64_t N1 = (int64_t)L.n1 * L.p + 1, N2 = (int64_t)L.n2 * L.p + 1;
    return I1 + N1 * (I2 + N2 * (int64_t)I3);
}

__global__ void k_skel_to_nodal(Layout L, const double* __restrict__ skel, double* __restrict__ nodal, int64_t N,
                                int k, int keep_con, uint32_t ns, int64_t rs) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < L.Ns; s += (int64_t)gridDim.x * blockDim.x) {
        bool con;
        const int64_t g = skel_nodal_index(L, s, &con);
        for (int r = 0; r < k; ++r) nodal[(int64_t)r * N + g] = (con && !keep_con) ? 0.0 : skel[s * ns + r * rs];
    }
}

__global__ void k_mask_nodes(Layout L, double* __restrict__ x, int k, int keep) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < L.Ns; s += (int64_t)gridDim.x * blockDim.x) {
        int I1, I2, I3;
        bool con;
        skeleton_node(L, s, &I1, &I2, &I3, &con);
        if (con != (keep == KEEP_CONSTRAINED))
            for (int r = 0; r < k; ++r) x[s * k + r] = 0.0;
    }
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

__global__ void k_nodal_to_skel(Layout L, const double* __restrict__ nodal, double* __restrict__ skel, int64_t N,
                                int k) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < L.Ns; s += (int64_t)gridDim.x * blockDim.x) {
        bool con;
        const int64_t g = skel_nodal_index(L, s, &con);
        for (int r = 0; r < k; ++r) skel[s * k + r] = nodal[(int64_t)r * N + g];
    }
}

static int grid_for(int64_t n, int threads) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_skel_to_nodal(const Layout& L, const double* skel, double* nodal, int64_t N, int k,
                                int keep_con, hipStream_t st, SkelStride sk) {
    sk = skel_stride(sk, k);
    hipLaunchKernelGGL(k_skel_to_nodal, dim3(grid_for(L.Ns, 256)), dim3(256), 0, st, L, skel, nodal, N, k,
                       keep_con, sk.ns, sk.rs);
    return hipGetLastError();
}

hipError_t launch_mask_nodes(const Layout& L, double* x, int k, int keep, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_nodes, dim3(grid_for(L.Ns, 256)), dim3(256), 0, st, L, x, k, keep);
    return hipGetLastError();
}

hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n, 256)), dim3(256), 0, st, y, x, a, n);
    return hipGetLastError();
}

hipError_t launch_nodal_to_skel(const Layout& L, const double* nodal, double* skel, int64_t N, int k,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_nodal_to_skel, dim3(grid_for(L.Ns, 256)), dim3(256), 0, st, L, nodal, skel, N, k);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fill and convert.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T* __restrict__ x, int64_t n, T val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = val;
}

template <typename T>
hipError_t launch_fill(T* x, int64_t n, T val, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256)), dim3(256), 0, st, x, n, val);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ in, Tout* __restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (Tout)in[i];
}

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);

// out[s*k + r] = active[r] ? (Tout)in[s*k + r] : 0   (residual hand-off of iterative refinement)
template <typename Tin, typename Tout>
__global__ void k_convert_masked(const Tin* __restrict__ in, Tout* __restrict__ out, int64_t n, int k,
                                 const int* __restrict__ active) {
    const int64_t len = n / k;  // [k][len], RHS-major
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = active[i / len] ? (Tout)in[i] : (Tout)0;
}

hipError_t launch_convert_masked(const double* in, float* out, int64_t n, int k, const int* active, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert_masked<double, float>), dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n, k,
                       active);
    return hipGetLastError();
}

// x += (double) d
__global__ void k_add_mixed(double* __restrict__ x, const float* __restrict__ d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += (double)d[i];
}

hipError_t launch_add_mixed(double* x, const float* d, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_mixed, dim3(grid_for(n, 256)), dim3(256), 0, st, x, d, n);
    return hipGetLastError();
}
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// Conjugate-gradient vector kernels on RHS-major multivectors [k][N_s]: block
// (x, r) of a grid (vec_blocks(k), k) works on right-hand side r, nodes
// x*256 + t + m*256*vec_blocks(k); its sums are formed in a fixed order.
// ---------------------------------------------------------------------------

int vec_blocks(int k) { return std::max(1, kVecBlocks / k); }

// Block sums of NQ quantities (all threads of the block belong to one RHS):
// partials[(q * gridDim.x + blockIdx.x) * k + blockIdx.y].
template <int NQ>
__device__ inline void block_partials(double (&acc)[NQ], int k, double* __restrict__ partials) {
    __shared__ double sh[NQ][4];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = wave_sum(acc[q]);
    if ((t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[q][t >> 6] = acc[q];
    }
    __syncthreads();
    if (t < NQ) {
        const double s = sh[t][0] + sh[t][1] + sh[t][2] + sh[t][3];
        partials[((int64_t)t * gridDim.x + blockIdx.x) * k + blockIdx.y] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(const T* __restrict__ b, T* __restrict__ q0,
                                                 const T* __restrict__ pinv, T* __restrict__ r, T* __restrict__ p,
                                                 int64_t Ns, int k, double* __restrict__ partials, int keep_p) {
    const int64_t off = (int64_t)blockIdx.y * Ns, stride = (int64_t)gridDim.x * blockDim.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < Ns; s += stride) {
        const int64_t idx = off + s;
        const T bv = b[idx];
        T rv = bv;
        if (q0) {
            rv = bv - q0[idx];
            q0[idx] = (T)0;  // leaves q zeroed for the first operator application
        }
        const T z = pinv[s] * rv;
        r[idx] = rv;
        if (!keep_p) p[idx] = (T)0;
        acc[0] += (double)rv * (double)z;
        acc[1] += (double)rv * (double)rv;
        acc[2] += (double)bv * (double)bv;
    }
    block_partials<3>(acc, k, partials);
}

template <typename T>
hipError_t launch_cg_init(const T* b, T* q0, const T* pinv, T* r, T* p, int64_t Ns, int k, double* partials,
                          hipStream_t st, bool keep_p) {
    hipLaunchKernelGGL(k_cg_init<T>, dim3(vec_blocks(k), k), dim3(256), 0, st, b, q0, pinv, r, p, Ns, k, partials,
                       keep_p ? 1 : 0);
    return hipGetLastError();
}
template hipError_t launch_cg_init<double>(const double*, double*, const double*, double*, double*, int64_t, int,
                                           double*, hipStream_t, bool);
template hipError_t launch_cg_init<float>(const float*, float*, const float*, float*, float*, int64_t, int, double*,
                                          hipStream_t, bool);

// One block of B = k * floor(256/k) threads: thread t sums RHS t mod k over
// the parts t/k, t/k + B/k, ... (all loads of a thread issued together).  For
// k a power of two up to 64 the B/k sums of one RHS are combined inside each
// wave by a fixed xor-shuffle tree and the waves' sums in wave order; otherwise
// a fixed-shape shared-memory tree adds them.  Then the CG scalar step per RHS.
constexpr int kReduceThreads = 256;

__global__ __launch_bounds__(kReduceThreads) void k_cg_reduce(const double* __restrict__ partials, int64_t nparts,
                                                              int nq, int k, CgState s, int mode) {
    __shared__ double sh[3][kReduceThreads];
    const int t = threadIdx.x, r = t % k, j = t / k, npb = blockDim.x / k;
    constexpr int U = 16;
    // per-RHS state read before anything is written, so that no load waits on a store
    const bool rz_mode = mode == RED_RZ || mode == RED_RZ_DEFER;
    int act = 0, its = 0, stall = 0;
    double rho = 0.0, bb = 0.0, tol2 = 0.0, rrb = 0.0, alpha_now = 0.0;
    if (t < k) {
        act = s.active[t];
        its = s.iters[t];
        rho = s.rho[t];
        bb = s.bb[t];
        tol2 = s.tol2[0];
        if (rz_mode) {
            rrb = s.rrb[t];
            stall = s.stall[t];
        }
        if (mode == RED_RZ_DEFER) alpha_now = s.alpha[t];
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t m0 = j; m0 < nparts; m0 += (int64_t)U * npb) {
        double v[3][U];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t m = m0 + (int64_t)u * npb;
                v[q][u] = (q < nq && m < nparts) ? partials[((int64_t)q * nparts + m) * k + r] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[q] += v[q][u];
    }
    const bool pow2 = k <= 64 && (k & (k - 1)) == 0;
    if (pow2) {
        // lanes l and l ^ off (off >= k, a multiple of k) hold the same RHS
        for (int off = 32; off >= k; off >>= 1) {
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] += __shfl_xor(acc[q], off, 64);
        }
        const int lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
        if (lane < k) {
#pragma unroll
            for (int q = 0; q < 3; ++q) sh[q][wv * k + lane] = acc[q];
        }
        __syncthreads();
        if (t < k) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double sum = sh[q][t];
                for (int w = 1; w < nw; ++w) sum += sh[q][w * k + t];
                acc[q] = sum;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) sh[q][t] = acc[q];
        __syncthreads();
        int P = 1;
        while (P < npb) P <<= 1;
        for (int w = P >> 1; w > 0; w >>= 1) {
            if (j < w && j + w < npb) {
#pragma unroll
                for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + w * k];
            }
            __syncthreads();
        }
        if (t < k) {
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = sh[q][t];
        }
    }
    if (t < k) {
        const double t0 = acc[0], t1 = acc[1], t2 = acc[2];
        if (mode == RED_INIT || mode == RED_INIT_KEEP) {
            const double rz = t0 + (s.rz_extra ? s.rz_extra[r] : 0.0), rr = t1, b2 = t2;
            s.rho[r] = rz;
            s.rr[r] = rr;
            s.bb[r] = b2;
            s.iters[r] = 0;
            s.alpha[r] = 0.0;
            // continued direction: the first step takes p = z + (r.z / rho_old) p_old,
            // rho_old the r.z that formed p_old (kept at convergence); a fresh
            // start has p = 0
            const bool cont = mode == RED_INIT_KEEP && rho > 0.0 && isfinite(rho) && isfinite(rz);
            s.beta[r] = cont ? rz / rho : 0.0;
            const bool bad = !isfinite(rr) || !isfinite(rz);
            s.status[r] = bad ? -5 : 0;
            s.active[r] = bad ? 0 : ((rr > tol2 * b2) ? 1 : 0);
            s.rrb[r] = rr;
            s.stall[r] = 0;
            if (s.xa) s.xa[r] = 0.0;
        } else if (mode == RED_PQ) {
            const double pq = t0;
            s.pq[r] = pq;
            double alpha = 0.0;
            if (act) {
                if (!isfinite(pq)) {
                    s.status[r] = -5;
                    s.active[r] = 0;
                } else if (!(pq > 0.0)) {
                    s.status[r] = -4;
                    s.active[r] = 0;
                } else {
                    alpha = rho / pq;
                }
            }
            s.alpha[r] = alpha;
        } else {  // RED_RZ, RED_RZ_DEFER
            const double rz = t0 + (s.rz_extra ? s.rz_extra[r] : 0.0), rr = t1;
            double beta = 0.0;
            if (act) {
                s.iters[r] = its + 1;
                // a deferring step leaves alpha p to the next step or the flush
                if (s.xa) s.xa[r] = mode == RED_RZ_DEFER ? alpha_now : 0.0;
                s.rr[r] = rr;
                if (!isfinite(rr) || !isfinite(rz)) {
                    s.status[r] = -5;
                    s.active[r] = 0;
                } else if (rr <= tol2 * bb) {
                    s.active[r] = 0;
                } else {
                    double rrb_new;
                    int stall_new;
                    if (cg_stalled(rr, rrb, stall, s.window, &rrb_new, &stall_new)) {
                        s.active[r] = 0;
                    } else {
                        beta = rz / rho;
                        s.rho[r] = rz;
                    }
                    s.rrb[r] = rrb_new;
                    s.stall[r] = stall_new;
                }
            }
            s.beta[r] = beta;
        }
    }
}

hipError_t launch_cg_reduce(const double* partials, int64_t nparts, int nq, int k, CgState s, int mode,
                            hipStream_t st) {
    if (k < 1 || k > kReduceThreads || nq < 1 || nq > 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(k * (kReduceThreads / k)), 0, st, partials, nparts, nq, k, s,
                       mode);
    return hipGetLastError();
}

// First stage of the p.q reduction over the element energies [n_e][k]: block
// b sums the elements of its contiguous range, every RHS in a fixed order
// (thread groups of k lanes take every G-th element, then the G group sums in
// group order), into out [gridDim.x][k].  The one-workgroup k_cg_reduce then
// reads these partials instead of all n_e k energies (one workgroup reading
// 1.8 MB took 68 us at 24^3 elements, 16 RHS).
constexpr int kEnergyThreads = 256;

__global__ __launch_bounds__(kEnergyThreads) void k_energy_partials(const double* __restrict__ energy,
                                                                    int64_t n_e, int k, double* __restrict__ out) {
    __shared__ double sh[kEnergyThreads];
    const int G = kEnergyThreads / k;  // thread groups of k lanes
    const int t = threadIdx.x, r = t % k, g = t / k;
    const int64_t chunk = (n_e + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * chunk;
    const int64_t e1 = e0 + chunk < n_e ? e0 + chunk : n_e;
    double acc = 0.0;
    if (g < G)
        for (int64_t e = e0 + g; e < e1; e += G) acc += energy[e * k + r];
    sh[t] = acc;
    __syncthreads();
    if (t < k) {
        double sum = 0.0;
        for (int q = 0; q < G; ++q) sum += sh[q * k + t];
        out[(int64_t)blockIdx.x * k + t] = sum;
    }
}

hipError_t launch_energy_pq(const double* energy, int64_t n_e, int k, double* epart, CgState s, hipStream_t st) {
    if (k < 1 || k > kEnergyThreads) return hipErrorInvalidValue;
    const int nb = (int)(n_e < kEnergyBlocks ? n_e : kEnergyBlocks);
    if (nb < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_partials, dim3(nb), dim3(kEnergyThreads), 0, st, energy, n_e, k, epart);
    return launch_cg_reduce(epart, nb, 1, k, s, RED_PQ, st);
}

// q of node n of RHS rhs: the slot sum for nodes whose rows went into slots
// (edges and vertices, faces too with face_slots), else q itself, which the
// caller clears for the next operator application (cg_q_clear).
template <typename T, bool SLOTS>
__device__ inline T cg_q(const T* __restrict__ q, const T* __restrict__ qs, int64_t qlen, const Layout& L, int rhs,
                         int64_t idx, int64_t n, int face_slots) {
    if constexpr (SLOTS) {
        if (face_slots || n >= L.oEx) return slot_sum(L, qs + (size_t)rhs * qlen, (uint32_t)n);
    }
    return q[idx];
}
template <bool SLOTS>
__device__ inline bool cg_q_clear(const Layout& L, int64_t n, int face_slots) {
    return !SLOTS || (!face_slots && n < L.oEx);
}

template <typename T, bool SLOTS, bool PFORMED = false, int XM = CG_X_NOW>
__global__ __launch_bounds__(256) void k_cg_step(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                 T* __restrict__ q, const T* __restrict__ pinv, int64_t Ns, int k,
                                                 CgState s, double* __restrict__ partials, const T* __restrict__ qs,
                                                 int64_t qlen, Layout L, int fsl) {
    static_assert(XM == CG_X_NOW || !PFORMED, "deferred x updates need the previous direction, which p_formed overwrites");
    const int rhs = blockIdx.y;
    const int64_t off = (int64_t)rhs * Ns, stride = (int64_t)gridDim.x * blockDim.x;
    const T alpha = (T)s.alpha[rhs];
    const T beta = (T)s.beta[rhs];
    // A stopped right-hand side keeps x, r and p; its q is not read again (the
    // apply skips it) and its partial sums are ignored.
    if (s.active[rhs] == 0) return;
    // the length of the previous (deferring) step, whose direction p holds
    const T xa = XM == CG_X_FLUSH ? (T)s.xa[rhs] : (T)0;
    double acc[2] = {0.0, 0.0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < Ns; n += stride) {
        const int64_t idx = off + n;
        T rv = r[idx];
        const T qv = cg_q<T, SLOTS>(q, qs, qlen, L, rhs, idx, n, fsl);
        const T pn = pinv[n];
        if (cg_q_clear<SLOTS>(L, n, fsl)) q[idx] = (T)0;  // q is accumulated from zero by the next apply
        T pv;
        if constexpr (PFORMED) {
            pv = p[idx];  // formed before the apply (two-level preconditioner)
            x[idx] += alpha * pv;
        } else {
            const T pold = p[idx];
            pv = fmadd(beta, pold, pn * rv);  // the direction the apply used
            p[idx] = pv;
            if constexpr (XM == CG_X_NOW) x[idx] += alpha * pv;
            if constexpr (XM == CG_X_FLUSH) x[idx] += fmadd(xa, pold, alpha * pv);
        }
        rv -= alpha * qv;
        r[idx] = rv;
        const T z = pn * rv;
        acc[0] += (double)rv * (double)z;
        acc[1] += (double)rv * (double)rv;
    }
    block_partials<2>(acc, k, partials);
}

template <typename T, int XM>
hipError_t launch_cg_step_x(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, CgState s, double* partials,
                            const T* qs, int64_t qlen, const Layout& L, int face_slots, hipStream_t st) {
    if (qs)
        hipLaunchKernelGGL((k_cg_step<T, true, false, XM>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q,
                           pinv, Ns, k, s, partials, qs, qlen, L, face_slots);
    else
        hipLaunchKernelGGL((k_cg_step<T, false, false, XM>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q,
                           pinv, Ns, k, s, partials, qs, qlen, L, face_slots);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_step(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, CgState s, double* partials,
                          const T* qs, int64_t qlen, const Layout& L, int face_slots, hipStream_t st, bool p_formed,
                          int x_mode) {
    if (x_mode != CG_X_NOW && (p_formed || !s.xa)) return hipErrorInvalidValue;
    if (x_mode == CG_X_DEFER)
        return launch_cg_step_x<T, CG_X_DEFER>(x, r, p, q, pinv, Ns, k, s, partials, qs, qlen, L, face_slots, st);
    if (x_mode == CG_X_FLUSH)
        return launch_cg_step_x<T, CG_X_FLUSH>(x, r, p, q, pinv, Ns, k, s, partials, qs, qlen, L, face_slots, st);
    if (p_formed) {
        if (qs)
            hipLaunchKernelGGL((k_cg_step<T, true, true>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q, pinv,
                               Ns, k, s, partials, qs, qlen, L, face_slots);
        else
            hipLaunchKernelGGL((k_cg_step<T, false, true>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q, pinv,
                               Ns, k, s, partials, qs, qlen, L, face_slots);
        return hipGetLastError();
    }
    if (qs)
        hipLaunchKernelGGL((k_cg_step<T, true>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q, pinv, Ns, k, s,
                           partials, qs, qlen, L, face_slots);
    else
        hipLaunchKernelGGL((k_cg_step<T, false>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, r, p, q, pinv, Ns, k,
                           s, partials, qs, qlen, L, face_slots);
    return hipGetLastError();
}
template hipError_t launch_cg_step<double>(double*, double*, double*, double*, const double*, int64_t, int, CgState,
                                           double*, const double*, int64_t, const Layout&, int, hipStream_t, bool,
                                           int);
template hipError_t launch_cg_step<float>(float*, float*, float*, float*, const float*, int64_t, int, CgState, double*,
                                          const float*, int64_t, const Layout&, int, hipStream_t, bool, int);

template <typename T>
__global__ __launch_bounds__(256) void k_cg_x_flush(T* __restrict__ x, const T* __restrict__ p, int64_t Ns,
                                                    const double* __restrict__ xa) {
    const int rhs = blockIdx.y;
    const T a = (T)xa[rhs];
    if (a == (T)0) return;
    const int64_t off = (int64_t)rhs * Ns, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < Ns; n += stride) x[off + n] += a * p[off + n];
}

// Clears xa in a second launch: every block of a RHS reads it before any clears it.
__global__ void k_cg_xa_clear(double* __restrict__ xa, int k) {
    if ((int)threadIdx.x < k) xa[threadIdx.x] = 0.0;
}

template <typename T>
hipError_t launch_cg_x_flush(T* x, const T* p, int64_t Ns, int k, CgState s, hipStream_t st) {
    if (!s.xa || k < 1 || k > kMaxRhs) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_cg_x_flush<T>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, p, Ns, s.xa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg_xa_clear, dim3(1), dim3(k), 0, st, s.xa, k);
    return hipGetLastError();
}
template hipError_t launch_cg_x_flush<double>(double*, const double*, int64_t, int, CgState, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void k_cg_x_flush_parity(T* __restrict__ x, const T* __restrict__ p, int64_t Ns,
                                                           const int* __restrict__ iters,
                                                           const double* __restrict__ alpha0) {
    const int rhs = blockIdx.y;
    if ((iters[rhs] & 1) == 0) return;
    const T a = (T)alpha0[rhs];
    const int64_t off = (int64_t)rhs * Ns, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < Ns; n += stride) x[off + n] += a * p[off + n];
}

template <typename T>
hipError_t launch_cg_x_flush_parity(T* x, const T* p, int64_t Ns, int k, const int* iters, const double* alpha0,
                                    hipStream_t st) {
    if (!iters || !alpha0 || k < 1 || k > kMaxRhs) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_cg_x_flush_parity<T>), dim3(vec_blocks(k), k), dim3(256), 0, st, x, p, Ns, iters, alpha0);
    return hipGetLastError();
}
template hipError_t launch_cg_x_flush_parity<double>(double*, const double*, int64_t, int, const int*, const double*,
                                                     hipStream_t);
template hipError_t launch_cg_x_flush_parity<float>(float*, const float*, int64_t, int, const int*, const double*,
                                                    hipStream_t);
template hipError_t launch_cg_x_flush<float>(float*, const float*, int64_t, int, CgState, hipStream_t);

int fused_step_blocks(int k) { return std::max(1, 256 / k); }

// The CG step with p.q completed by every block from the element energies
// (blocks of kFusedStepThreads threads, fused_step_blocks(k) per RHS: few
// blocks, so that each apply workgroup's later reduction of their partials
// stays small).
template <typename T, bool SLOTS, int XM>
__global__ __launch_bounds__(kFusedStepThreads) void k_cg_step_fused(T* __restrict__ x, T* __restrict__ r,
                                                                     T* __restrict__ p, T* __restrict__ q,
                                                                     const T* __restrict__ pinv, int64_t Ns, int k,
                                                                     CgFuse f, double* __restrict__ partials,
                                                                     const T* __restrict__ qs, int64_t qlen, Layout L,
                                                                     int fsl) {
    constexpr int NT = kFusedStepThreads;
    __shared__ double s_red[2 * (NT / 64)];
    const int rhs = blockIdx.y;
    if (!f.act[rhs]) return;  // stopped (its state is already carried by the apply)
    const int64_t off = (int64_t)rhs * Ns, stride = (int64_t)gridDim.x * NT;
    double pq[1];
    block_sums<NT, 1>(f.energy + rhs, 0, f.n_e, k, s_red, pq);
    bool act;
    const T alpha = (T)cg_pq_complete(f, rhs, pq[0], blockIdx.x == 0 && threadIdx.x == 0, &act);
    // a stopped RHS keeps x, r and p; its q and partial sums are not read again
    if (!act) return;
    const T beta = (T)f.beta[rhs];
    // the previous (deferring) step's length: its slot is not written in this launch
    const T xa = XM == CG_X_FLUSH ? (T)f.alpha_prev[rhs] : (T)0;
    double acc[2] = {0.0, 0.0};
    auto node = [&](int64_t n, T rv, T qv, T pn, T pold) __attribute__((always_inline)) {
        const int64_t idx = off + n;
        if (cg_q_clear<SLOTS>(L, n, fsl)) q[idx] = (T)0;  // q is accumulated from zero by the next apply
        const T pv = fmadd(beta, pold, pn * rv);  // the direction the apply used
        p[idx] = pv;
        if constexpr (XM == CG_X_NOW) x[idx] += alpha * pv;
        if constexpr (XM == CG_X_FLUSH) x[idx] += fmadd(xa, pold, alpha * pv);
        rv -= alpha * qv;
        r[idx] = rv;
        const T z = pn * rv;
        acc[0] += (double)rv * (double)z;
        acc[1] += (double)rv * (double)rv;
    };
    for (int64_t n = (int64_t)blockIdx.x * NT + threadIdx.x; n < Ns; n += stride) {
        const int64_t idx = off + n;
        node(n, r[idx], cg_q<T, SLOTS>(q, qs, qlen, L, rhs, idx, n, fsl), pinv[n], p[idx]);
    }
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) acc[qq] = wave_sum(acc[qq]);
    __syncthreads();  // s_red is free
    if ((threadIdx.x & 63) == 0) {
        s_red[threadIdx.x >> 6] = acc[0];
        s_red[NT / 64 + (threadIdx.x >> 6)] = acc[1];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double sum = 0.0;
        for (int w = 0; w < NT / 64; ++w) sum += s_red[threadIdx.x * (NT / 64) + w];
        partials[((int64_t)threadIdx.x * gridDim.x + blockIdx.x) * k + rhs] = sum;
    }
}

template <typename T, int XM>
hipError_t launch_cg_step_fused_x(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, const CgFuse& f,
                                  double* partials, const T* qs, int64_t qlen, const Layout& L, int face_slots,
                                  hipStream_t st) {
    if (qs)
        hipLaunchKernelGGL((k_cg_step_fused<T, true, XM>), dim3(fused_step_blocks(k), k), dim3(kFusedStepThreads), 0,
                           st, x, r, p, q, pinv, Ns, k, f, partials, qs, qlen, L, face_slots);
    else
        hipLaunchKernelGGL((k_cg_step_fused<T, false, XM>), dim3(fused_step_blocks(k), k), dim3(kFusedStepThreads), 0,
                           st, x, r, p, q, pinv, Ns, k, f, partials, qs, qlen, L, face_slots);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_step_fused(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, const CgFuse& f,
                                double* partials, const T* qs, int64_t qlen, const Layout& L, int face_slots,
                                hipStream_t st) {
    if (f.x_mode == CG_X_DEFER)
        return launch_cg_step_fused_x<T, CG_X_DEFER>(x, r, p, q, pinv, Ns, k, f, partials, qs, qlen, L, face_slots,
                                                     st);
    if (f.x_mode == CG_X_FLUSH) {
        if (!f.alpha_prev) return hipErrorInvalidValue;
        return launch_cg_step_fused_x<T, CG_X_FLUSH>(x, r, p, q, pinv, Ns, k, f, partials, qs, qlen, L, face_slots,
                                                     st);
    }
    return launch_cg_step_fused_x<T, CG_X_NOW>(x, r, p, q, pinv, Ns, k, f, partials, qs, qlen, L, face_slots, st);
}
template hipError_t launch_cg_step_fused<double>(double*, double*, double*, double*, const double*, int64_t, int,
                                                 const CgFuse&, double*, const double*, int64_t, const Layout&, int,
                                                 hipStream_t);
template hipError_t launch_cg_step_fused<float>(float*, float*, float*, float*, const float*, int64_t, int,
                                                const CgFuse&, double*, const float*, int64_t, const Layout&, int,
                                                hipStream_t);

// out[c][r] = in[r][c] for an R x C row-major array, 32 x 32 tiles through LDS;
// a one-dimensional grid of tiles (tile t: rows (t / tc) * 32, columns
// (t mod tc) * 32, tc = ceil(C / 32)).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ in, T* __restrict__ out, int64_t R,
                                                   int64_t C, int64_t tc) {
    __shared__ T tile[32][33];
    const int64_t tid = blockIdx.x;
    const int64_t r0 = tid / tc * 32, c0 = tid % tc * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int64_t rr = r0 + i, cc = c0 + tx;
        if (rr < R && cc < C) tile[i][tx] = in[rr * C + cc];
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int64_t cc = c0 + i, rr = r0 + tx;
        if (rr < R && cc < C) out[cc * R + rr] = tile[tx][i];
    }
}

template <typename T>
hipError_t launch_transpose(const T* in, T* out, int64_t R, int64_t C, hipStream_t st) {
    if (R <= 0 || C <= 0) return hipSuccess;
    const int64_t tr = (R + 31) / 32, tc = (C + 31) / 32;
    if (tr * tc > (int64_t(1) << 24)) return hipErrorInvalidValue;  // work-items stay below 2^32
    hipLaunchKernelGGL(k_transpose<T>, dim3((unsigned)(tr * tc)), dim3(256), 0, st, in, out, R, C, tc);
    return hipGetLastError();
}
template hipError_t launch_transpose<double>(const double*, double*, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<float>(const float*, float*, int64_t, int64_t, hipStream_t);

}  // namespace semcond

namespace semcond {

// ---------------------------------------------------------------------------
// Assembled GLL-lumped mass M_G = R (J_e W(x)W(x)W) R^T, a diagonal (Sec. 3).
// With J_e = prod_a h_a/2 it factorises per axis: M_G(I) = prod_a m_a(I_a),
// m_a(I) = sum over the elements e_a containing I of (h_a(e_a)/2) w_{I - e_a p}.
// ---------------------------------------------------------------------------

__device__ inline double axis_mass(const double* h, int n, int p, const double* w, int I) {
    const int e = I / p, loc = I - e * p;
    double m = 0.0;
    if (e < n) m += 0.5 * h[e] * w[loc];
    if (loc == 0 && e > 0) m += 0.5 * h[e - 1] * w[p];
    return m;
}

__global__ void k_nodal_mass(Geo g, const double* __restrict__ w, double* __restrict__ mass) {
    const Layout& L = g.L;
    const int p = L.p;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1, N3 = (int64_t)L.n3 * p + 1;
    const int64_t N = N1 * N2 * N3;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * blockDim.x) {
        const int I1 = (int)(idx % N1);
        const int64_t r = idx / N1;
        const int I2 = (int)(r % N2), I3 = (int)(r / N2);
        mass[idx] = axis_mass(g.hx, L.n1, p, w, I1) * axis_mass(g.hy, L.n2, p, w, I2) * axis_mass(g.hz, L.n3, p, w, I3);
    }
}

hipError_t launch_nodal_mass(const Geo& g, const double* w, double* mass, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_nodal_mass, dim3(grid_for(N, 256)), dim3(256), 0, st, g, w, mass);
    return hipGetLastError();
}

// out[r][I] = in[r][I] * M_G(I)  (or / M_G(I) when inverse), nodal [k][N].
__global__ void k_mass_apply(Geo g, const double* __restrict__ w, const double* __restrict__ in,
                             double* __restrict__ out, int k, int inverse) {
    const Layout& L = g.L;
    const int p = L.p;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1, N3 = (int64_t)L.n3 * p + 1;
    const int64_t N = N1 * N2 * N3;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * blockDim.x) {
        const int I1 = (int)(idx % N1);
        const int64_t rr = idx / N1;
        const int I2 = (int)(rr % N2), I3 = (int)(rr / N2);
        const double m = axis_mass(g.hx, L.n1, p, w, I1) * axis_mass(g.hy, L.n2, p, w, I2) *
                         axis_mass(g.hz, L.n3, p, w, I3);
        for (int r = 0; r < k; ++r) {
            const int64_t o = (int64_t)r * N + idx;
            out[o] = inverse ? in[o] / m : in[o] * m;
        }
    }
}

hipError_t launch_mass_apply(const Geo& g, const double* w, const double* in, double* out, int64_t N, int k,
                             int inverse, hipStream_t st) {
    hipLaunchKernelGGL(k_mass_apply, dim3(grid_for(N, 256)), dim3(256), 0, st, g, w, in, out, k, inverse);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Element gradients of a loss L(u) through H_G u = M_G f (adjoint a = H_G^-1 dL/du):
//   grad[e][m] = dL/dd_{e,m} = -a_e^T A_m u_e (m = 0..3), grad[e][4] = dL/dlambda_e = J_e grad[e][0],
//    A_0 = M(x)M(x)M, A_1 = M(x)M(x)K, A_2 = M(x)K(x)M,
//   A_3 = K(x)M(x)M (Sec. 3, eq. helmholtz_operator), summed over the k right-hand
//   sides; u and a are nodal [k][N].  One workgroup per element; each thread
//   handles whole 1D lines of the element.
// ---------------------------------------------------------------------------

// PER_RHS: grad[e][m][r] = -a_{e,r}^T A_m u_{e,r} for every right-hand side r
// ([n_e][4][k]) instead of the sum over r with the lambda column.
template <bool PER_RHS>
__global__ __launch_bounds__(256) void k_element_grads(Geo g, const double* __restrict__ w, const double* __restrict__ K,
                                                       const double* __restrict__ u, const double* __restrict__ a,
                                                       int64_t N, int k, double* __restrict__ grad) {
    __shared__ double red[4][256];
    const Layout& L = g.L;
    const int p = L.p, n = p + 1;
    const int64_t N1 = (int64_t)L.n1 * p + 1, N2 = (int64_t)L.n2 * p + 1;
    const int64_t e = blockIdx.x;
    int e1, e2, e3;
    elem_index(L, e, &e1, &e2, &e3);
    const int64_t base = (int64_t)e1 * p + N1 * ((int64_t)e2 * p + N2 * (int64_t)e3 * p);
    const int64_t stride[3] = {1, N1, N1 * N2};  // node stride along i, j, k
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < k; ++r) {
        const double* ur = u + (int64_t)r * N + base;
        const double* ar = a + (int64_t)r * N + base;
        // mass term: sum w_i w_j w_k a u over the element's nodes
        for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
            const int i = idx % n, j = (idx / n) % n, kk = idx / (n * n);
            const int64_t off = i + N1 * (j + N2 * (int64_t)kk);
            acc[0] += w[i] * w[j] * w[kk] * ar[off] * ur[off];
        }
        // stiffness terms: lines along axis ax, weighted by w of the two other indices
        for (int t = threadIdx.x; t < 3 * n * n; t += blockDim.x) {
            const int ax = t / (n * n), l = t % (n * n), s1 = l / n, s2 = l % n;
            int64_t lb;
            double wt;
            if (ax == 0) { lb = N1 * (s2 + N2 * (int64_t)s1); wt = w[s1] * w[s2]; }        // (k, j) fixed
            else if (ax == 1) { lb = s2 + N1 * N2 * (int64_t)s1; wt = w[s1] * w[s2]; }     // (k, i) fixed
            else { lb = s2 + N1 * (int64_t)s1; wt = w[s1] * w[s2]; }                        // (j, i) fixed
            const int64_t st = stride[ax];
            double s = 0.0;
            for (int i = 0; i < n; ++i) {
                double ku = 0.0;
                for (int i2 = 0; i2 < n; ++i2) ku += K[i * n + i2] * ur[lb + i2 * st];
                s += ar[lb + i * st] * ku;
            }
            acc[1 + ax] += wt * s;
        }
        if constexpr (PER_RHS) {
            // fixed-order block sum of this right-hand side's four terms
            __syncthreads();  // red free from the previous right-hand side
            for (int m = 0; m < 4; ++m) red[m][threadIdx.x] = acc[m];
            __syncthreads();
            for (int s = 128; s > 0; s >>= 1) {
                if ((int)threadIdx.x < s)
                    for (int m = 0; m < 4; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x < 4) grad[(e * 4 + threadIdx.x) * k + r] = -red[threadIdx.x][0];
            for (int m = 0; m < 4; ++m) acc[m] = 0.0;
        }
    }
    if constexpr (!PER_RHS) {
        for (int m = 0; m < 4; ++m) red[m][threadIdx.x] = acc[m];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
                for (int m = 0; m < 4; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x < 4) grad[e * 5 + threadIdx.x] = -red[threadIdx.x][0];
        if (threadIdx.x == 4) grad[e * 5 + 4] = -red[0][0] * elem_jacobian(g, e1, e2, e3);  // d d0 / d lambda_e = J_e
    }
}

hipError_t launch_element_grads(const Geo& g, const double* w, const double* K, const double* u, const double* a,
                                int64_t N, int k, double* grad, bool per_rhs, hipStream_t st) {
    const int64_t ne = (int64_t)g.L.n1 * g.L.n2 * g.L.n3;
    if (per_rhs)
        hipLaunchKernelGGL(k_element_grads<true>, dim3((unsigned)ne), dim3(256), 0, st, g, w, K, u, a, N, k, grad);
    else
        hipLaunchKernelGGL(k_element_grads<false>, dim3((unsigned)ne), dim3(256), 0, st, g, w, K, u, a, N, k, grad);
    return hipGetLastError();
}

}  // namespace semcond
