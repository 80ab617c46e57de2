// Two-level preconditioner for the BT conjugate gradients (optional): the
// diagonal of the transformed condensed operator (Sec. 8's block
// preconditioner) plus a coarse correction on the space of trilinear
// functions of the element mesh, P A_0^-1 P^T.  The coarse unknowns are the
// values at the element vertices; P interpolates them trilinearly to the
// skeleton nodes and maps to the transformed basis, where on a face node
// (s1, s2) the weight of a corner is t_a(s1) t_b(s2), on an edge node t_a(m)
// and on a vertex 1, with t_0 = S^-1 (1 - x)/2 and t_1 = S^-1 (1 + x)/2 at the
// interior GLL nodes.  A_0 is the trilinear finite-element matrix with the
// element metrics d_e (exactly P^T H^ P for lambda = 0, where trilinear
// functions are discretely harmonic), factored once by Cholesky and inverted,
// so that each coarse solve is one matrix product streaming A_0^-1 once.
// The multigrid direction of the paper's outlook (Sec. 9) in two levels.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"
#include "layout.h"

namespace semcond {

namespace {

__device__ inline int64_t vertex_id(const Layout& L, int vx, int vy, int vz) {
    return vx + (int64_t)(L.n1 + 1) * (vy + (int64_t)(L.n2 + 1) * vz);
}

// Corner vertices of skeleton entity containing node n, and the node's local
// position: kind 0 face (4 corners, weights t_a(s1) t_b(s2) with corner c =
// a + 2 b... see below), 1 edge (2 corners, t_a(m)), 2 vertex (itself).
struct NodeCorners {
    int kind;
    int s1, s2;  // face: local slot; edge: s1 = node along the edge
    int64_t v[4];
};

// Decode skeleton node n.  Face corners are listed as v[a_slow + 2 a_fast]
// with a_slow selecting t(s1), a_fast t(s2); edge corners v[a], weight t_a(s1).
__device__ inline void node_corners(const Layout& L, int64_t n, NodeCorners* c) {
    const int NI = L.NI;
    const int64_t NI2 = (int64_t)NI * NI;
    if (n < L.oEx) {
        c->kind = 0;
        int64_t f = n / NI2;
        const int loc = (int)(n - f * NI2);
        c->s1 = loc / NI;
        c->s2 = loc % NI;
        const int64_t nFx = (L.oFy - L.oFx) / NI2, nFy = (L.oFz - L.oFy) / NI2;
        if (f < nFx) {  // Fx[e3][e2][fx], slot (k, j): slow = k, fast = j
            const int fx = (int)(f % (L.n1 + 1));
            const int64_t rr = f / (L.n1 + 1);
            const int e2 = (int)(rr % L.n2), e3 = (int)(rr / L.n2);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) c->v[a + 2 * b] = vertex_id(L, fx, e2 + b, e3 + a);
        } else if (f < nFx + nFy) {  // Fy[e3][fy][e1], slot (k, i)
            f -= nFx;
            const int e1 = (int)(f % L.n1);
            const int64_t rr = f / L.n1;
            const int fy = (int)(rr % (L.n2 + 1)), e3 = (int)(rr / (L.n2 + 1));
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) c->v[a + 2 * b] = vertex_id(L, e1 + b, fy, e3 + a);
        } else {  // Fz[fz][e2][e1], slot (j, i)
            f -= nFx + nFy;
            const int e1 = (int)(f % L.n1);
            const int64_t rr = f / L.n1;
            const int e2 = (int)(rr % L.n2), fz = (int)(rr / L.n2);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) c->v[a + 2 * b] = vertex_id(L, e1 + b, e2 + a, fz);
        }
        return;
    }
    if (n < L.oV) {
        c->kind = 1;
        if (n < L.oEy) {  // Ex[ez][ey][e1], along x1
            const int64_t t = n - L.oEx, g = t / NI;
            c->s1 = (int)(t % NI);
            const int e1 = (int)(g % L.n1);
            const int64_t rr = g / L.n1;
            const int ey = (int)(rr % (L.n2 + 1)), ez = (int)(rr / (L.n2 + 1));
            c->v[0] = vertex_id(L, e1, ey, ez);
            c->v[1] = vertex_id(L, e1 + 1, ey, ez);
        } else if (n < L.oEz) {  // Ey[ez][e2][ex], along x2
            const int64_t t = n - L.oEy, g = t / NI;
            c->s1 = (int)(t % NI);
            const int ex = (int)(g % (L.n1 + 1));
            const int64_t rr = g / (L.n1 + 1);
            const int e2 = (int)(rr % L.n2), ez = (int)(rr / L.n2);
            c->v[0] = vertex_id(L, ex, e2, ez);
            c->v[1] = vertex_id(L, ex, e2 + 1, ez);
        } else {  // Ez[e3][ey][ex], along x3
            const int64_t t = n - L.oEz, g = t / NI;
            c->s1 = (int)(t % NI);
            const int ex = (int)(g % (L.n1 + 1));
            const int64_t rr = g / (L.n1 + 1);
            const int ey = (int)(rr % (L.n2 + 1)), e3 = (int)(rr / (L.n2 + 1));
            c->v[0] = vertex_id(L, ex, ey, e3);
            c->v[1] = vertex_id(L, ex, ey, e3 + 1);
        }
        return;
    }
    c->kind = 2;
    c->v[0] = n - L.oV;
}

constexpr int kCoarseThreads = 256;

}  // namespace

// r0[rhs][vmap[v]] += sum over the skeleton nodes of v's entities of weight x
// r(node); faces one wave each, edges and vertices one thread each.  r0 must be
// zeroed first.  r: value (node, rhs) at node + rhs * rs (RHS-major).
template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_restrict_faces(Layout L, const double* __restrict__ tw,
                                                                          const int* __restrict__ vmap, int n0,
                                                                          const T* __restrict__ r, int64_t rs,
                                                                          const int* __restrict__ act,
                                                                          double* __restrict__ r0) {
    const int rhs = blockIdx.y;
    if (act && !act[rhs]) return;
    const int NI = L.NI;
    const int64_t NI2 = (int64_t)NI * NI, nfaces = L.oEx / NI2;
    const int lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * (kCoarseThreads / 64) + (threadIdx.x >> 6);
    if (f >= nfaces) return;  // the whole wave leaves
    const double* t0 = tw;
    const double* t1 = tw + NI;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = lane; q < NI2; q += 64) {
        const int s1 = q / NI, s2 = q % NI;
        const double rv = (double)r[f * NI2 + q + rhs * rs];
        const double a0 = t0[s1] * rv, a1 = t1[s1] * rv;
        acc[0] += a0 * t0[s2];
        acc[1] += a1 * t0[s2];
        acc[2] += a0 * t1[s2];
        acc[3] += a1 * t1[s2];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = wave_sum(acc[m]);
    if (lane == 0) {
        NodeCorners c;
        node_corners(L, f * NI2, &c);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int iv = vmap[c.v[m]];
            if (iv >= 0) atomic_add(&r0[(int64_t)rhs * n0 + iv], acc[m]);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_restrict_rest(Layout L, const double* __restrict__ tw,
                                                                         const int* __restrict__ vmap, int n0,
                                                                         const T* __restrict__ r, int64_t rs,
                                                                         const int* __restrict__ act,
                                                                         double* __restrict__ r0) {
    const int rhs = blockIdx.y;
    if (act && !act[rhs]) return;
    const int NI = L.NI;
    const int64_t nedges = (L.oV - L.oEx) / NI, nvert = L.Ns - L.oV;
    const int64_t g = (int64_t)blockIdx.x * kCoarseThreads + threadIdx.x;
    if (g < nedges) {
        const int64_t base = L.oEx + g * NI;
        double a0 = 0.0, a1 = 0.0;
        for (int m = 0; m < NI; ++m) {
            const double rv = (double)r[base + m + rhs * rs];
            a0 += tw[m] * rv;
            a1 += tw[NI + m] * rv;
        }
        NodeCorners c;
        node_corners(L, base, &c);
        const int i0 = vmap[c.v[0]], i1 = vmap[c.v[1]];
        if (i0 >= 0) atomic_add(&r0[(int64_t)rhs * n0 + i0], a0);
        if (i1 >= 0) atomic_add(&r0[(int64_t)rhs * n0 + i1], a1);
    } else if (g < nedges + nvert) {
        const int64_t v = g - nedges;
        const int iv = vmap[v];
        if (iv >= 0) atomic_add(&r0[(int64_t)rhs * n0 + iv], (double)r[L.oV + v + rhs * rs]);
    }
}

template <typename T>
hipError_t launch_coarse_restrict(const Layout& L, const double* tw, const int* vmap, int n0, const T* r, int k,
                                  const int* act, double* r0, hipStream_t st) {
    const int NI = L.NI;
    const int64_t nfaces = L.oEx / ((int64_t)NI * NI);
    const int64_t nrest = (L.oV - L.oEx) / NI + (L.Ns - L.oV);
    if (nfaces > 0) {
        const int64_t b = (nfaces + kCoarseThreads / 64 - 1) / (kCoarseThreads / 64);
        hipLaunchKernelGGL(k_coarse_restrict_faces<T>, dim3((unsigned)b, (unsigned)k), dim3(kCoarseThreads), 0, st, L,
                           tw, vmap, n0, r, L.Ns, act, r0);
    }
    const int64_t b2 = (nrest + kCoarseThreads - 1) / kCoarseThreads;
    hipLaunchKernelGGL(k_coarse_restrict_rest<T>, dim3((unsigned)b2, (unsigned)k), dim3(kCoarseThreads), 0, st, L, tw,
                       vmap, n0, r, L.Ns, act, r0);
    return hipGetLastError();
}
template hipError_t launch_coarse_restrict<double>(const Layout&, const double*, const int*, int, const double*, int,
                                                   const int*, double*, hipStream_t);
template hipError_t launch_coarse_restrict<float>(const Layout&, const double*, const int*, int, const float*, int,
                                                  const int*, double*, hipStream_t);

// out[rhs] = sum_v a[rhs][v] b[rhs][v] (r0 . A_0^-1 r0), one block per RHS.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_dot(const double* __restrict__ a,
                                                               const double* __restrict__ b, int n0,
                                                               double* __restrict__ out) {
    __shared__ double s_red[kCoarseThreads / 64];
    const int rhs = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n0; i += kCoarseThreads)
        acc += a[(int64_t)rhs * n0 + i] * b[(int64_t)rhs * n0 + i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kCoarseThreads / 64; ++w) s += s_red[w];
        out[rhs] = s;
    }
}

hipError_t launch_coarse_dot(const double* a, const double* b, int n0, int k, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_coarse_dot, dim3(k), dim3(kCoarseThreads), 0, st, a, b, n0, out);
    return hipGetLastError();
}

// Copy the lower triangle of the n x n column-major matrix A into its upper
// triangle (A symmetric afterwards).
__global__ void k_symmetrize_lower(double* __restrict__ A, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = idx / n, row = idx - col * n;
        if (row < col) A[idx] = A[row * n + col];  // (row, col) upper <- (col, row) lower
    }
}

hipError_t launch_symmetrize_lower(double* A, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_symmetrize_lower, dim3(4096), dim3(256), 0, st, A, n);
    return hipGetLastError();
}

// Direction update of the two-level CG: p = P^-1 r + P z0 + beta p for the
// active RHS (P z0: the coarse correction interpolated to the node; 0 at
// vertices that are not coarse unknowns).  RHS-major vectors; one thread per
// skeleton node for all RHS (the node's corners and weights are decoded once).
template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_pupd(Layout L, const double* __restrict__ tw,
                                                                const int* __restrict__ vmap, int n0,
                                                                const double* __restrict__ z0,
                                                                const T* __restrict__ pinv, const T* __restrict__ r,
                                                                T* __restrict__ p, int k, CgState s) {
    const int NI = L.NI;
    const double* t0 = tw;
    const double* t1 = tw + NI;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < L.Ns; n += (int64_t)gridDim.x * blockDim.x) {
        NodeCorners c;
        node_corners(L, n, &c);
        double w[4] = {0.0, 0.0, 0.0, 0.0};
        int iv[4] = {-1, -1, -1, -1};
        if (c.kind == 0) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    iv[a + 2 * b] = vmap[c.v[a + 2 * b]];
                    w[a + 2 * b] = (a ? t1 : t0)[c.s1] * (b ? t1 : t0)[c.s2];
                }
        } else if (c.kind == 1) {
            iv[0] = vmap[c.v[0]];
            iv[1] = vmap[c.v[1]];
            w[0] = t0[c.s1];
            w[1] = t1[c.s1];
        } else {
            iv[0] = vmap[c.v[0]];
            w[0] = 1.0;
        }
        const T pn = pinv[n];
        for (int rhs = 0; rhs < k; ++rhs) {
            if (s.active[rhs] == 0) continue;
            const double* zr = z0 + (int64_t)rhs * n0;
            double cv = 0.0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                if (iv[m] >= 0) cv += w[m] * zr[iv[m]];
            const int64_t idx = (int64_t)rhs * L.Ns + n;
            p[idx] = fmadd((T)s.beta[rhs], p[idx], pn * r[idx] + (T)cv);
        }
    }
}

template <typename T>
hipError_t launch_coarse_pupd(const Layout& L, const double* tw, const int* vmap, int n0, const double* z0,
                              const T* pinv, const T* r, T* p, int k, CgState s, hipStream_t st) {
    int64_t b = (L.Ns + kCoarseThreads - 1) / kCoarseThreads;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(k_coarse_pupd<T>, dim3((unsigned)b), dim3(kCoarseThreads), 0, st, L, tw, vmap, n0, z0, pinv,
                       r, p, k, s);
    return hipGetLastError();
}
template hipError_t launch_coarse_pupd<double>(const Layout&, const double*, const int*, int, const double*,
                                               const double*, const double*, double*, int, CgState, hipStream_t);
template hipError_t launch_coarse_pupd<float>(const Layout&, const double*, const int*, int, const double*,
                                              const float*, const float*, float*, int, CgState, hipStream_t);

// z0 = Ainv r0 for the symmetric n0 x n0 column-major Ainv and up to 16 RHS
// (r0, z0 [k][n0]; z0 zeroed first): workgroup (x, y) takes rows x*256 ..
// x*256 + 255 (one per thread) and the column range y of kCoarseSplit, streams
// its columns of Ainv once (coalesced: the rows of a column are contiguous) and
// reads the RHS values from an LDS copy of each 64-column chunk; partial sums
// are added into z0 atomically.
constexpr int kCoarseSplit = 8;
constexpr int kCoarseChunk = 64;

__global__ __launch_bounds__(kCoarseThreads) void k_coarse_gemv16(const double* __restrict__ Ainv, int n0,
                                                                  const double* __restrict__ r0, int k,
                                                                  double* __restrict__ z0) {
    __shared__ double sR[kCoarseChunk][16];
    const int64_t row = (int64_t)blockIdx.x * kCoarseThreads + threadIdx.x;
    const int64_t per = ((int64_t)n0 + kCoarseSplit - 1) / kCoarseSplit;
    const int64_t j_begin = blockIdx.y * per;
    const int64_t j_end = j_begin + per < n0 ? j_begin + per : n0;
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    for (int64_t j0 = j_begin; j0 < j_end; j0 += kCoarseChunk) {
        __syncthreads();  // sR free from the previous chunk
        for (int t = threadIdx.x; t < kCoarseChunk * 16; t += kCoarseThreads) {
            const int jj = t % kCoarseChunk, r = t / kCoarseChunk;
            sR[jj][r] = (r < k && j0 + jj < j_end) ? r0[(int64_t)r * n0 + j0 + jj] : 0.0;
        }
        __syncthreads();
        if (row < n0) {
            const int nj = (int)(j_end - j0 < kCoarseChunk ? j_end - j0 : kCoarseChunk);
            for (int jj = 0; jj < nj; ++jj) {
                const double a = Ainv[(j0 + jj) * n0 + row];
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[r] += a * sR[jj][r];
            }
        }
    }
    if (row < n0) {
        for (int r = 0; r < k && r < 16; ++r) atomic_add(&z0[(int64_t)r * n0 + row], acc[r]);
    }
}

hipError_t launch_coarse_gemv(const double* Ainv, int n0, const double* r0, int k, double* z0, hipStream_t st) {
    const unsigned bx = (unsigned)((n0 + kCoarseThreads - 1) / kCoarseThreads);
    for (int r = 0; r < k; r += 16) {
        const int kk = k - r < 16 ? k - r : 16;
        hipLaunchKernelGGL(k_coarse_gemv16, dim3(bx, kCoarseSplit), dim3(kCoarseThreads), 0, st, Ainv, n0,
                           r0 + (int64_t)r * n0, kk, z0 + (int64_t)r * n0);
    }
    return hipGetLastError();
}

}  // namespace semcond
