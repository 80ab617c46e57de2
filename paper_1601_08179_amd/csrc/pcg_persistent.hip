// BT conjugate gradients (Sec. 8) for k right-hand sides in one persistent,
// cooperative launch.
//
// Every iteration runs three phases separated by grid-wide barriers:
//   A  q = H~^ p on all elements (apply_element.h), per-RHS energies p.q;
//   B  alpha = rho / p.q, x += alpha p, r -= alpha q, q = 0, partial r.z, r.r;
//   C  beta, convergence per RHS, p = z + beta p  (z = P~^-1 r, never stored).
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

// Grid barrier on bar[0] (arrival count) and bar[32] (generation, separate
// cache line).  Returns false when the wait bound was exceeded or another
// workgroup raised the error flag.
__device__ inline bool grid_barrier(unsigned* bar, int* err, unsigned spin_limit, int* s_ok) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* count = bar;
        unsigned* gen = bar + 32;
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(count, 1u);
        int ok = 1;
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(gen, 1u);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > spin_limit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 0;
                    break;
                }
            }
        }
        if (!ok) atomicExch(err, 1);
        *s_ok = ok;
    }
    __syncthreads();
    __threadfence();
    return *s_ok != 0;
}

// out[r] = sum over workgroups b of part[(q*G + b)*k + r], in a fixed order.
template <int WG>
__device__ inline void reduce_partials(const double* part, int q, int k, double* s_red, double* out) {
    const int t = threadIdx.x, G = gridDim.x, r = t % k, j = t / k, npb = WG / k;
    double acc = 0.0;
#pragma unroll 4
    for (int b = j; b < G; b += npb) acc += part[((int64_t)q * G + b) * k + r];
    s_red[t] = acc;
    __syncthreads();
    int P = 1;
    while (P < npb) P <<= 1;
    for (int w = P >> 1; w > 0; w >>= 1) {
        if (j < w && j + w < npb) s_red[t] += s_red[t + w * k];
        __syncthreads();
    }
    if (t < k) out[t] = s_red[t];
    __syncthreads();
}

// Per-workgroup partial of one quantity: s_red holds one value per thread
// (thread t belongs to RHS t mod k); writes part[(q*G + b)*k + r].
template <int WG>
__device__ inline void write_partial(double* s_red, int k, double* part, int q) {
    const int t = threadIdx.x, j = t / k, npb = WG / k;
    __syncthreads();
    int P = 1;
    while (P < npb) P <<= 1;
    for (int w = P >> 1; w > 0; w >>= 1) {
        if (j < w && j + w < npb) s_red[t] += s_red[t + w * k];
        __syncthreads();
    }
    if (t < k) part[((int64_t)q * gridDim.x + blockIdx.x) * k + t] = s_red[t];
    __syncthreads();
}

template <typename T, int NI, int S>
__global__ __launch_bounds__(S * apply_threads(NI)) void k_pcg_persistent(PcgArgs<T> P) {
    constexpr int NT = apply_threads(NI);
    constexpr int WG = S * NT;
    constexpr int KM = kPersistMaxK;
    __shared__ ApplySmem<T, NI> sm[S];
    __shared__ double s_en[S][KM];
    __shared__ double s_rho[KM], s_alpha[KM], s_beta[KM], s_bb[KM], s_rr[KM], s_tot[2][KM];
    __shared__ int s_act[KM], s_iters[KM], s_status[KM];
    __shared__ double s_red[WG], s_red2[WG];
    __shared__ int s_flag, s_ok;

    const int t = threadIdx.x, sub = t / NT, lt = t - sub * NT;
    const int k = P.k, G = gridDim.x, b = blockIdx.x;
    const int rfix = t % k, npb = WG / k;
    if (t < k) {
        s_rho[t] = P.rho[t];
        s_rr[t] = P.rr[t];
        s_bb[t] = P.bb[t];
        s_act[t] = P.active[t];
        s_iters[t] = P.iters[t];
        s_status[t] = P.status[t];
    }
    const double tol2 = P.tol2;
    __syncthreads();
    const int64_t per_round = (int64_t)G * S;
    const int64_t rounds = (P.n_e + per_round - 1) / per_round;

    for (int it = 0; it < P.max_iter; ++it) {
        if (t == 0) {
            int any = 0;
            for (int r = 0; r < k; ++r) any |= s_act[r];
            s_flag = any;
        }
        __syncthreads();
        if (!s_flag) break;

        // ---- A: q = H~^ p, energies p.q
        if (lt < k) s_en[sub][lt] = 0.0;
        __syncthreads();
        for (int64_t m = 0; m < rounds; ++m) {
            const int64_t e = (m * G + b) * S + sub;
            const bool live = e < P.n_e;
            apply_element<T, NI>(P.A, live ? e : 0, sm[sub], s_en[sub], lt, live);
        }
        if (t < k) {
            double s = 0.0;
            for (int g = 0; g < S; ++g) s += s_en[g][t];
            P.part[((int64_t)0 * G + b) * k + t] = s;
        }
        if (!grid_barrier(P.bar, P.err, P.spin_limit, &s_ok)) return;

        // ---- B: alpha, x and r updates
        reduce_partials<WG>(P.part, 0, k, s_red, s_tot[0]);
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
        {
            const T alpha = (T)s_alpha[rfix];
            const bool act = s_act[rfix] != 0;
            double arz = 0.0, arr = 0.0;
            for (int64_t n = (int64_t)b * npb + t / k; n < P.Ns; n += (int64_t)G * npb) {
                const int64_t idx = n * k + rfix;
                T rv = P.r[idx];
                const T qv = P.q[idx];
                P.q[idx] = (T)0;
                if (act) {
                    P.x[idx] += alpha * P.p[idx];
                    rv -= alpha * qv;
                    P.r[idx] = rv;
                }
                const T z = P.pinv[n] * rv;
                arz += (double)rv * (double)z;
                arr += (double)rv * (double)rv;
            }
            s_red[t] = arz;
            s_red2[t] = arr;
            write_partial<WG>(s_red, k, P.part, 1);
            write_partial<WG>(s_red2, k, P.part, 2);
        }
        if (!grid_barrier(P.bar, P.err, P.spin_limit, &s_ok)) return;

        // ---- C: beta, convergence, direction
        reduce_partials<WG>(P.part, 1, k, s_red, s_tot[0]);
        reduce_partials<WG>(P.part, 2, k, s_red, s_tot[1]);
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
                } else {
                    s_beta[t] = rz / s_rho[t];
                    s_rho[t] = rz;
                }
            } else {
                s_beta[t] = 0.0;
            }
        }
        __syncthreads();
        if (s_act[rfix]) {
            const T beta = (T)s_beta[rfix];
            for (int64_t n = (int64_t)b * npb + t / k; n < P.Ns; n += (int64_t)G * npb) {
                const int64_t idx = n * k + rfix;
                P.p[idx] = P.pinv[n] * P.r[idx] + beta * P.p[idx];
            }
        }
        if (!grid_barrier(P.bar, P.err, P.spin_limit, &s_ok)) return;
    }
    if (b == 0 && t < k) {
        P.rho[t] = s_rho[t];
        P.rr[t] = s_rr[t];
        P.active[t] = s_act[t];
        P.iters[t] = s_iters[t];
        P.status[t] = s_status[t];
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
