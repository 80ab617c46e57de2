// Persistent cooperative BT conjugate-gradient kernel (see pcg_persistent.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace semcond {

constexpr int kPersistMaxK = 32;  // right-hand sides of one persistent launch

template <typename T>
struct PcgArgs {
    ApplyArgs<T> A;  // operator: A.u = p, A.v = q, A.k = k, A.energy = nullptr
    T* x;
    T* r;
    T* p;
    T* q;            // zero on entry; zeroed again after every use
    const T* pinv;   // [N_s] inverse preconditioner diagonal
    int64_t Ns, n_e;
    int k;
    double* part;    // [3][grid][k] workgroup partials
    // CG state (device, per RHS), read at start and written back at exit
    double* rho;
    double* rr;
    const double* bb;
    int* active;
    int* iters;
    int* status;
    double tol2;
    int max_iter;
    unsigned* bar;   // grid barrier words (bar[0] count, bar[32] generation), zero on first use
    int* err;        // set when a barrier wait exceeded spin_limit
    unsigned spin_limit;
};

// Whether (n_I, S, k) has a compiled persistent kernel: n_I <= 15, S = 1 or
// the largest group count for n_I, k <= kPersistMaxK dividing the workgroup.
bool persist_supported(int NI, int S, int k);
int persist_threads(int NI, int S);
// Largest co-resident grid for (n_I, S) on the current device (0 if unknown).
template <typename T>
int persist_max_grid(int NI, int S);
template <typename T>
hipError_t launch_pcg_persistent(const PcgArgs<T>& P, int NI, int S, int grid, hipStream_t st);

}  // namespace semcond
