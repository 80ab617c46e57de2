// Condensed Helmholtz operator in the transformed basis, v~ = R H~^_L R^T u~
// (Sec. 6, Table 2).  One workgroup per element (several elements, one per lane
// group, for n_I <= 5) and right-hand side; the element bodies are in
// apply_element.h.

#include <hip/hip_runtime.h>

#include "apply_element.h"
#include "cg_device.h"

namespace semcond {

// Workgroups are dispatched to the 8 XCDs of the chip in turn (workgroup b to
// XCD b mod 8), each XCD with its own L2.  In the CG applies element blocks are
// handed out so that every XCD works on one contiguous range of elements:
// neighbours, which share faces, edges and vertices, then mostly share an L2
// too (measured 1-2 % faster solves; the standalone apply, whose rows all go
// through atomics, measured up to 7 % slower with it and keeps the plain order).
// A bijection of [0, nb): XCD x takes nb / 8 (+1 for x < nb mod 8) consecutive
// blocks.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
    const uint32_t x = b & 7u, i = b >> 3, per = nb >> 3, rem = nb & 7u;
    return x * per + (x < rem ? x : rem) + i;
}

// Waves per SIMD the compiler is asked to fit: the FP32 cube kernels at
// 9 <= n_I <= 11 hold 80-88 VGPRs, i.e. 5 waves; capping them at 80 (6 waves,
// at most one spilled value) measured 5 % faster at p = 12 with 16 RHS.  FP64
// kernels forced to more waves spill and ran slower, and so would the fused
// CG kernels (FZ).
template <typename T, int NI, bool FZ>
constexpr int apply_waves() { return sizeof(T) == 4 && !FZ && NI >= 9 && NI <= 11 ? 6 : 1; }

// FZ (with DIR): the previous CG step's r.z is completed in the kernel
// (A.fz), a separate instantiation so that plain launches keep their registers.
template <typename T, int NI, bool DIR, bool FZ>
__global__ __launch_bounds__(apply_threads(NI)) __attribute__((amdgpu_waves_per_eu(apply_waves<T, NI, FZ>())))
void k_apply_tpt(ApplyArgs<T> A, int64_t n_elem) {
    constexpr int NT = apply_threads(NI);
    constexpr bool CUBE = NI <= 15;
    const double* beta = A.dir_beta;
    if constexpr (DIR && FZ && !CUBE) {
        // CG direction with the previous step's r.z completed here: every
        // workgroup reduces the step's partial sums for all right-hand sides
        // in one fixed order (the cube form does this inside its gather)
        __shared__ double s_beta[kMaxRhs];
        __shared__ double s_red[2 * (NT / 64)];
        {
            const bool writer = blockIdx.x == 0 && threadIdx.x == 0;
            bool any = false;
            for (int r = 0; r < A.k; ++r) {
                double t[2];
                block_sums<NT, 2>(A.fz.part + r, (int64_t)A.fz.nsb * A.k, A.fz.nsb, A.k, s_red, t);
                bool still;
                const double b = cg_rz_complete(A.fz, r, t[0], t[1], writer, &still);
                any |= still;
                if (threadIdx.x == 0) s_beta[r] = b;
            }
            // nothing to apply once every RHS of the workgroup has stopped (the
            // step ignores the energies of stopped RHS); the same in all threads
            if (!any) return;
            __syncthreads();
            beta = s_beta;
        }
    }
    if constexpr (CUBE) {
        // workgroup (x, y): elements e_begin + x*E .. + E - 1, right-hand side y
        constexpr int E = apply_pack(NI);
        __shared__ ApplySmem<T, NI> sm[E];
        const uint32_t eb = DIR ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
        apply_elements_cube<T, NI, DIR, true, E, FZ>(A, A.e_begin + (int64_t)eb * E, 1, 1, A.e_begin + n_elem,
                                                     blockIdx.y, 1, sm, nullptr, threadIdx.x, beta);
    } else {
        __shared__ ApplySmem<T, NI> sm;
        const uint32_t eb = DIR ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
        apply_element<T, NI, DIR>(A, (int64_t)eb + A.e_begin, sm, nullptr, threadIdx.x, true, beta);
    }
}

// Grid of the apply: for n_I <= 15 one workgroup per apply_pack(n_I) elements
// and right-hand side (measured faster on gfx950 than workgroups that walk
// several items), else one per element.  Element counts stay below 2^31 (the
// skeleton is larger than the element count and N_s k < 2^31); k <= 256.
template <int NI>
static dim3 apply_grid(int64_t n_elem, int k) {
    if (NI > 15) return dim3((unsigned)n_elem);
    constexpr int E = apply_pack(NI);
    return dim3((unsigned)((n_elem + E - 1) / E), (unsigned)k);
}

template <typename T>
hipError_t launch_apply_tpt(const ApplyArgs<T>& a, int64_t n_elem, hipStream_t st) {
    const int NI = a.g.L.NI;
    if (n_elem <= 0) return hipSuccess;
#define CASE(N)                                                                                                    \
    case N:                                                                                                        \
        if (a.dir_r && a.fz.part)                                                                                  \
            hipLaunchKernelGGL((k_apply_tpt<T, N, true, true>), apply_grid<N>(n_elem, a.k), dim3(apply_threads(N)), \
                               0, st, a, n_elem);                                                                  \
        else if (a.dir_r)                                                                                          \
            hipLaunchKernelGGL((k_apply_tpt<T, N, true, false>), apply_grid<N>(n_elem, a.k),                      \
                               dim3(apply_threads(N)), 0, st, a, n_elem);                                          \
        else                                                                                                       \
            hipLaunchKernelGGL((k_apply_tpt<T, N, false, false>), apply_grid<N>(n_elem, a.k),                     \
                               dim3(apply_threads(N)), 0, st, a, n_elem);                                          \
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
