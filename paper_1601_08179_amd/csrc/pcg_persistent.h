// Persistent cooperative BT conjugate-gradient kernel (see pcg_persistent.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace semcond {

constexpr int kPersistMaxK = 32;  // right-hand sides of one persistent launch
// Grid barrier words: kBarGroups group counters, a top counter, the generation
// and the error flag, each kBarSlot unsigned words (256 B) apart.
constexpr int kBarSlot = 64;
constexpr int kBarGroups = 64;
constexpr int kBarWords = (kBarGroups + 3) * kBarSlot;

template <typename T>
struct PcgArgs {
    ApplyArgs<T> A;  // operator: A.u = p, A.v = q, A.k = k, A.energy = nullptr, RHS-major strides
    // x, r, p, q: RHS-major [k][N_s]
    T* x;
    T* r;
    T* p;            // previous direction (0 with beta = 0 before the first step)
    T* q;            // zero on entry; zeroed again after every use
    const T* pinv;   // [N_s] inverse preconditioner diagonal
    int64_t Ns, n_e;
    int k;
    double* part;    // [3][grid][k] workgroup partials
    // CG state (device, per RHS), read at start and written back at exit
    double* rho;
    double* beta;
    double* rr;
    const double* bb;
    int* active;
    int* iters;
    int* status;
    double* rrb;     // stagnation state (see CgState), window <= 0: off
    int* stall;
    int window;
    double tol2;
    int max_iter;
    unsigned* bar;   // kBarWords grid barrier words, zero on first use
    int* err;        // set when a barrier wait exceeded spin_limit (own 256-B slot)
    unsigned spin_limit;
#ifdef SEMCOND_PCG_TRACE
    long long* trace;  // [kPcgTraceIters][4][grid] wall-clock stamps (instrumented builds only)
#endif
};

#ifdef SEMCOND_PCG_TRACE
constexpr int kPcgTraceIters = 16;
#endif

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
