// Condensed Helmholtz operator in the transformed basis, one workgroup per
// element: v~ = R H~^_L R^T u~ (Sec. 6, Table 2).  The element body is in
// apply_element.h.

#include <hip/hip_runtime.h>

#include "apply_element.h"

namespace semcond {

template <typename T, int NI, bool DIR>
__global__ __launch_bounds__(apply_threads(NI)) void k_apply_tpt(ApplyArgs<T> A) {
    __shared__ ApplySmem<T, NI> sm;
    apply_element<T, NI, DIR>(A, (int64_t)blockIdx.x + A.e_begin, sm, nullptr, threadIdx.x, true, A.dir_beta);
}

template <typename T>
hipError_t launch_apply_tpt(const ApplyArgs<T>& a, int64_t n_elem, hipStream_t st) {
    const int NI = a.g.L.NI;
    if (n_elem <= 0) return hipSuccess;
    dim3 grid((unsigned)n_elem);
#define CASE(N)                                                                                \
    case N:                                                                                    \
        if (a.dir_r)                                                                           \
            hipLaunchKernelGGL((k_apply_tpt<T, N, true>), grid, dim3(apply_threads(N)), 0, st, a); \
        else                                                                                   \
            hipLaunchKernelGGL((k_apply_tpt<T, N, false>), grid, dim3(apply_threads(N)), 0, st, a); \
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
