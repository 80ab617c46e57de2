// BT conjugate gradients (Sec. 8) for k right-hand sides in one persistent,
// cooperative launch.
//
// Every iteration runs two phases separated by grid-wide barriers:
//   A  p = beta p + z (z = P~^-1 r, formed at the gather, never stored),
//      q = H~^ p on all elements (apply_element.h), per-RHS energies p.q;
//   B  alpha = rho / p.q; on the workgroup's nodes p is formed again (bitwise
//      the same) and stored, x += alpha p, r -= alpha q, q = 0; partial r.z,
//      r.r; then beta and convergence per RHS.
// The scalars are reduced by every workgroup from the per-workgroup partials
// in one fixed order, so all workgroups take identical decisions (exit, per-RHS
// freeze) without further communication, and results do not depend on
// scheduling.  A workgroup holds S element groups of apply_threads(n_I)
// threads that work on S elements at once; the grid size G and S are the
// tunables.  The grid barrier spins with a bound: a workgroup that waits past
// the bound raises an error flag and leaves, and every other workgroup leaves
// at its next barrier, so a fault cannot hang the device.

#include <hip/hip_runtime.h>

#include "apply_element.h"
#include "pcg_persistent.h"

namespace semcond {

// Grid barrier, two levels: workgroups arrive on the counter of their group
// of gs consecutive workgroups; the last arrival of a group arrives on the top
// counter, and the last group bumps the generation that everyone waits on.
// Same-address atomics are executed one after another at the memory side, so
// the tree keeps every counter at no more than max(32, G/64) arrivals.
// Words live kBarSlot words (256 B) apart: bar[g * kBarSlot] group counters,
// bar[kBarGroups * kBarSlot] top counter, bar[(kBarGroups + 1) * kBarSlot]
// generation.  One thread per workgroup synchronises: the workgroup barrier
// orders the other waves' stores before its agent-scope release (the arrival
// increment; arrivals are acquire-release, so the chain of increments carries
// every workgroup's stores to the generation bump), and its agent-scope acquire
// after the wait is followed by a workgroup barrier.  The spin uses relaxed
// loads so that waiting workgroups do not invalidate the caches of those still
// working.  Returns false when the wait bound was exceeded or another
// workgroup raised the error flag.
__device__ inline bool grid_barrier(unsigned* bar, int* err, unsigned spin_limit, int* s_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned G = gridDim.x;
        const unsigned gs = max(32u, (G + kBarGroups - 1) / kBarGroups);
        const unsigned ng = (G + gs - 1) / gs;
        const unsigned grp = blockIdx.x / gs;
        const unsigned gsize = min(gs, G - grp * gs);
        unsigned* cnt = bar + grp * kBarSlot;
        unsigned* top = bar + kBarGroups * kBarSlot;
        unsigned* gen = bar + (kBarGroups + 1) * kBarSlot;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        bool released = false;
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == ng - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > spin_limit) {
                    ok = 0;
                    break;
                }
                if ((spins & 63u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Store that is made coherent at device scope as it is written (through the
// XCD's L2), so the release at the next grid barrier has no dirty lines of the
// CG vectors to write back; every vector is re-read only after that barrier's
// acquire, which invalidates the L2 anyway.
template <typename T>
__device__ inline void store_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// out[q][r] = sum over workgroups b of part[(q*G + b)*k + r] for q < NQ, in a
// fixed order; every load of a thread is issued before the first add.
template <int WG, int NQ>
__device__ inline void reduce_partials(const double* part, int k, double (*s_red)[WG], double (*out)[kPersistMaxK]) {
    const int t = threadIdx.x, G = gridDim.x, r = t % k, j = t / k, npb = WG / k;
    constexpr int U = 4;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int b0 = j; b0 < G; b0 += U * npb) {
        double v[NQ][U];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = b0 + u * npb;
                v[q][u] = b < G ? part[((int64_t)q * G + b) * k + r] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[q] += v[q][u];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) s_red[q][t] = acc[q];
    __syncthreads();
    int P = 1;
    while (P < npb) P <<= 1;
    for (int w = P >> 1; w > 0; w >>= 1) {
        if (j < w && j + w < npb) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) s_red[q][t] += s_red[q][t + w * k];
        }
        __syncthreads();
    }
    if (t < k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q][t] = s_red[q][t];
    }
    __syncthreads();
}

#ifdef SEMCOND_PCG_TRACE
#define PCG_STAMP(ph)                                \
    if (P.trace && t == 0 && it < kPcgTraceIters) \
        P.trace[((int64_t)it * 4 + (ph)) * G + b] = wall_clock64();
#else
#define PCG_STAMP(ph)
#endif

template <typename T, int NI, int S>
__global__ __launch_bounds__(S * apply_threads(NI), 2) void k_pcg_persistent(PcgArgs<T> P) {
    constexpr int NT = apply_threads(NI);
    constexpr int WG = S * NT;
    constexpr int KM = kPersistMaxK;
    constexpr int U = 4;  // nodes per thread whose loads are issued together in phase B
    __shared__ ApplySmem<T, NI> sm[S];
    __shared__ double s_en[S][KM];
    __shared__ double s_rho[KM], s_alpha[KM], s_beta[KM], s_bb[KM], s_rr[KM], s_tot[2][KM];
    __shared__ int s_act[KM], s_iters[KM], s_status[KM], s_stall[KM];
    __shared__ double s_rrb[KM];
    __shared__ double s_red[2][WG];
    __shared__ int s_flag, s_ok;

    const int t = threadIdx.x, sub = t / NT, lt = t - sub * NT;
    const int k = P.k, G = gridDim.x, b = blockIdx.x;
    const int npb = WG / k;
    if (t < k) {
        s_rho[t] = P.rho[t];
        s_beta[t] = P.beta[t];
        s_rr[t] = P.rr[t];
        s_bb[t] = P.bb[t];
        s_act[t] = P.active[t];
        s_iters[t] = P.iters[t];
        s_status[t] = P.status[t];
        s_rrb[t] = P.rrb[t];
        s_stall[t] = P.stall[t];
    }
    const double tol2 = P.tol2;
    __syncthreads();
    const int64_t per_round = (int64_t)G * S;
    const int64_t rounds = (P.n_e + per_round - 1) / per_round;
    const int64_t vstride = (int64_t)G * npb;

    for (int it = 0; it < P.max_iter; ++it) {
        if (t == 0) {
            int any = 0;
            for (int r = 0; r < k; ++r) any |= s_act[r];
            s_flag = any;
        }
        __syncthreads();
        if (!s_flag) break;
        PCG_STAMP(0)

        // ---- A: q = H~^ p with p = beta p + z formed at the gather, energies p.q
        if (lt < k) s_en[sub][lt] = 0.0;
        __syncthreads();
        apply_elements_cube<T, NI, true, false>(P.A, (int64_t)b * S + sub, (int64_t)G * S, rounds, P.n_e, 0,
                                                (uint32_t)k, &sm[sub], s_en[sub], lt, s_beta);
        if (t < k) {
            double s = 0.0;
            for (int g = 0; g < S; ++g) s += s_en[g][t];
            P.part[(int64_t)b * k + t] = s;
        }
        PCG_STAMP(1)
        if (!grid_barrier(P.bar, P.err, P.spin_limit, &s_ok)) return;

        // ---- B: alpha; p, x, r updates on this workgroup's nodes; r.z, r.r
        reduce_partials<WG, 1>(P.part, k, s_red, s_tot);
        if (t < k) {
            const double pq = s_tot[0][t];
            if (s_act[t]) {
                if (!isfinite(pq)) {
                    s_status[t] = -5;
                    s_act[t] = 0;
                    s_alpha[t] = 0.0;
                } else if (!(pq > 0.0)) {
                    s_status[t] = -4;
                    s_act[t] = 0;
                    s_alpha[t] = 0.0;
                } else {
                    s_alpha[t] = s_rho[t] / pq;
                }
            } else {
                s_alpha[t] = 0.0;
            }
        }
        __syncthreads();
        PCG_STAMP(2)
        {
            // RHS-major vectors: thread t works on RHS rb = t / npb, nodes
            // b*npb + jb + m*G*npb (consecutive threads, consecutive nodes)
            const int rb = t / npb, jb = t - rb * npb;
            const T alpha = (T)s_alpha[rb], beta = (T)s_beta[rb];
            const bool act = s_act[rb] != 0;
            const int64_t off = (int64_t)rb * P.Ns;
            double arz = 0.0, arr = 0.0;
            for (int64_t n0 = (int64_t)b * npb + jb; n0 < P.Ns; n0 += U * vstride) {
                T rv[U], qv[U], pv[U], xv[U], pn[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t n = n0 + u * vstride;
                    const bool in = n < P.Ns;
                    const int64_t idx = off + n;
                    rv[u] = in ? P.r[idx] : (T)0;
                    qv[u] = in ? P.q[idx] : (T)0;
                    pn[u] = in ? P.pinv[n] : (T)0;
                    pv[u] = in && act ? P.p[idx] : (T)0;
                    xv[u] = in && act ? P.x[idx] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t n = n0 + u * vstride;
                    if (n < P.Ns) {
                        const int64_t idx = off + n;
                        store_dev(P.q + idx, (T)0);
                        if (act) {
                            const T pd = fmadd(beta, pv[u], pn[u] * rv[u]);
                            store_dev(P.p + idx, pd);
                            store_dev(P.x + idx, xv[u] + alpha * pd);
                            rv[u] -= alpha * qv[u];
                            store_dev(P.r + idx, rv[u]);
                        }
                        const T z = pn[u] * rv[u];
                        arz += (double)rv[u] * (double)z;
                        arr += (double)rv[u] * (double)rv[u];
                    }
                }
            }
            s_red[0][t] = arz;
            s_red[1][t] = arr;
            __syncthreads();
            int Pw = 1;
            while (Pw < npb) Pw <<= 1;
            for (int w = Pw >> 1; w > 0; w >>= 1) {
                if (jb < w && jb + w < npb) {
                    s_red[0][t] += s_red[0][t + w];
                    s_red[1][t] += s_red[1][t + w];
                }
                __syncthreads();
            }
            if (jb == 0) {
                P.part[((int64_t)1 * G + b) * k + rb] = s_red[0][t];
                P.part[((int64_t)2 * G + b) * k + rb] = s_red[1][t];
            }
        }
        PCG_STAMP(3)
        if (!grid_barrier(P.bar, P.err, P.spin_limit, &s_ok)) return;

        // ---- beta and convergence per RHS
        reduce_partials<WG, 2>(P.part + (int64_t)G * k, k, s_red, s_tot);
        if (t < k) {
            const double rz = s_tot[0][t], rr = s_tot[1][t];
            if (s_act[t]) {
                s_iters[t] += 1;
                s_rr[t] = rr;
                if (!isfinite(rr) || !isfinite(rz)) {
                    s_status[t] = -5;
                    s_act[t] = 0;
                    s_beta[t] = 0.0;
                } else if (rr <= tol2 * s_bb[t]) {
                    s_act[t] = 0;
                    s_beta[t] = 0.0;
                } else if (cg_stalled(rr, s_rrb[t], s_stall[t], P.window, &s_rrb[t], &s_stall[t])) {
                    s_act[t] = 0;
                    s_beta[t] = 0.0;
                } else {
                    s_beta[t] = rz / s_rho[t];
                    s_rho[t] = rz;
                }
            } else {
                s_beta[t] = 0.0;
            }
        }
        __syncthreads();
    }
    if (b == 0 && t < k) {
        P.rho[t] = s_rho[t];
        P.beta[t] = s_beta[t];
        P.rr[t] = s_rr[t];
        P.active[t] = s_act[t];
        P.iters[t] = s_iters[t];
        P.status[t] = s_status[t];
        P.rrb[t] = s_rrb[t];
        P.stall[t] = s_stall[t];
    }
}

// Element groups per workgroup that are compiled for n_I.
constexpr int persist_smax(int NI) { return apply_threads(NI) == 64 ? 4 : (apply_threads(NI) == 128 ? 2 : 1); }

int persist_threads(int NI, int S) { return S * (NI * NI <= 64 ? 64 : ((NI * NI + 63) / 64) * 64); }

bool persist_supported(int NI, int S, int k) {
    if (NI < 1 || NI > 15 || k < 1 || k > kPersistMaxK) return false;
    const int NT = NI * NI <= 64 ? 64 : ((NI * NI + 63) / 64) * 64;
    const int smax = NT == 64 ? 4 : (NT == 128 ? 2 : 1);
    if (S != 1 && S != smax) return false;
    return (S * NT) % k == 0;
}

template <typename T, int NI, int S>
static hipError_t launch_one(const PcgArgs<T>& P, int grid, hipStream_t st) {
    void* args[] = {(void*)&P};
    return hipLaunchCooperativeKernel((const void*)k_pcg_persistent<T, NI, S>, dim3(grid),
                                      dim3(S * apply_threads(NI)), args, 0, st);
}

template <typename T, int NI, int S>
static int max_grid_one() {
    int nb = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_pcg_persistent<T, NI, S>,
                                                     S * apply_threads(NI), 0) != hipSuccess)
        return 0;
    return nb * cus;
}

#define PERSIST_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

template <typename T>
hipError_t launch_pcg_persistent(const PcgArgs<T>& P, int NI, int S, int grid, hipStream_t st) {
    switch (NI) {
#define X(N)                                                                   \
    case N:                                                                    \
        if (S == 1) return launch_one<T, N, 1>(P, grid, st);                   \
        if (S == persist_smax(N)) return launch_one<T, N, persist_smax(N)>(P, grid, st); \
        return hipErrorInvalidValue;
        PERSIST_CASES(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
int persist_max_grid(int NI, int S) {
    switch (NI) {
#define X(N)                                                            \
    case N:                                                             \
        if (S == 1) return max_grid_one<T, N, 1>();                     \
        if (S == persist_smax(N)) return max_grid_one<T, N, persist_smax(N)>(); \
        return 0;
        PERSIST_CASES(X)
#undef X
        default:
            return 0;
    }
}

template hipError_t launch_pcg_persistent<double>(const PcgArgs<double>&, int, int, int, hipStream_t);
template hipError_t launch_pcg_persistent<float>(const PcgArgs<float>&, int, int, int, hipStream_t);
template int persist_max_grid<double>(int, int);
template int persist_max_grid<float>(int, int);

}  // namespace semcond
