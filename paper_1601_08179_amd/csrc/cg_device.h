// Device side of the conjugate-gradient scalar logic (BT solver, Sec. 8): the
// per-right-hand-side completion of each reduction, shared by the reduction
// kernel and by the kernels that reduce their producer's partial sums
// themselves.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace semcond {

// Sums of NQ strided arrays, out[q] = sum of v[q * qstride + i * stride] for i
// in [0, n), over the NT threads of a workgroup in a fixed order (thread t:
// i = t, t + NT, ... in sequence, U loads per quantity in flight; then each wave by its
// shuffle tree, waves in index order).  Every thread receives the sums;
// s_red holds NQ * NT / 64 doubles.
template <int NT, int NQ, int U = 8>
__device__ inline void block_sums(const double* v, int64_t qstride, int64_t n, int64_t stride, double* s_red,
                                  double (&out)[NQ]) {
    const int t = threadIdx.x;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int64_t i0 = t; i0 < n; i0 += (int64_t)U * NT) {
        double x[NQ][U];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + (int64_t)u * NT;
                x[q][u] = i < n ? v[q * qstride + i * stride] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[q] += x[q][u];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = wave_sum(acc[q]);
    if constexpr (NT > 64) {
        __syncthreads();  // s_red free from any earlier use
        if ((t & 63) == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) s_red[q * (NT / 64) + (t >> 6)] = acc[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double sum = s_red[q * (NT / 64)];
#pragma unroll
            for (int w = 1; w < NT / 64; ++w) sum += s_red[q * (NT / 64) + w];
            acc[q] = sum;
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = acc[q];
}

// Completion of the r.z / r.r reduction of a step for RHS r (RED_RZ):
// iteration count, convergence on r.r <= tol^2 b.b (rho kept: the r.z that
// formed the last direction, which a continued solve divides by), else beta =
// r.z / rho and rho = r.z.  Reads the state of the previous iteration's slot (rho_prev,
// act_prev) and, when `store`, writes this iteration's slot and the per-RHS
// counters.  Returns beta (0 for a converged or stopped RHS); *still receives
// whether the RHS keeps iterating.
// Stagnation test of an inner solve of the iterative refinement: progress means
// r.r below a quarter of its value at the last progress (the residual norm
// halved), which resets the count; a right-hand side whose residual has not
// halved for `window` iterations stops (window <= 0: never).  FP32 recurrences
// cannot reduce the residual much below the operator's own rounding level,
// so without this test an inner tolerance below that level would keep the
// inner solve running to its iteration limit.
__device__ inline bool cg_stalled(double rr, double rrb_old, int stall_old, int window, double* rrb_new,
                                  int* stall_new) {
    if (rr < 0.25 * rrb_old) {
        *rrb_new = rr;
        *stall_new = 0;
        return false;
    }
    *rrb_new = rrb_old;
    *stall_new = stall_old + 1;
    return window > 0 && *stall_new >= window;
}

__device__ inline double cg_rz_complete(const CgFuse& f, int r, double rz, double rr, bool store, bool* still) {
    const int act = f.act_prev[r];
    const double rho = f.rho_prev[r];
    double beta = 0.0, rho_new = rho;
    int act_new = act, status = 0;
    double rrb = f.rrb_prev[r];
    int stall = f.stall_prev[r];
    if (act) {
        if (!isfinite(rr) || !isfinite(rz)) {
            status = -5;
            act_new = 0;
        } else if (rr <= f.tol2[0] * f.bb[r]) {
            act_new = 0;
        } else if (cg_stalled(rr, f.rrb_prev[r], f.stall_prev[r], f.window, &rrb, &stall)) {
            act_new = 0;
        } else {
            beta = rz / rho;
            rho_new = rz;
        }
    }
    *still = act_new != 0;
    if (store) {
        if (act) {
            f.iters[r] = f.iters[r] + 1;
            f.rr[r] = rr;
        }
        if (status) f.status[r] = status;
        f.rho[r] = rho_new;
        f.act[r] = act_new;
        f.beta[r] = beta;
        f.rrb[r] = rrb;
        f.stall[r] = stall;
        if (f.host_act) f.host_act[r] = f.epoch2 + act_new;
    }
    return beta;
}

// The state of a RHS that had stopped before this iteration, carried into this
// iteration's slot (what cg_rz_complete stores for it).
__device__ inline void cg_carry_stopped(const CgFuse& f, int r) {
    f.rho[r] = f.rho_prev[r];
    f.act[r] = 0;
    f.beta[r] = 0.0;
    f.rrb[r] = f.rrb_prev[r];
    f.stall[r] = f.stall_prev[r];
    if (f.host_act) f.host_act[r] = f.epoch2;
}

// Completion of p.q for RHS r (RED_PQ) on this iteration's slot: alpha =
// rho / p.q, breakdown on p.q <= 0 (status -4) or non-finite p.q (-5).  When
// `store`, writes pq, alpha and a breakdown's status and stop.  Returns alpha;
// *act receives whether the RHS is still iterating.
__device__ inline double cg_pq_complete(const CgFuse& f, int r, double pq, bool store, bool* act) {
    const int a = f.act[r];
    double alpha = 0.0;
    int status = 0;
    if (a) {
        if (!isfinite(pq))
            status = -5;
        else if (!(pq > 0.0))
            status = -4;
        else
            alpha = f.rho[r] / pq;
    }
    *act = a && !status;
    if (store) {
        f.pq[r] = pq;
        f.alpha[r] = alpha;
        if (status) {
            f.status[r] = status;
            f.act[r] = 0;
            if (f.host_act) f.host_act[r] = f.epoch2;
        }
    }
    return alpha;
}

}  // namespace semcond
