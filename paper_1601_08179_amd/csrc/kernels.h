// Kernel launchers (host-callable) and their argument structs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace semcond {

// Layout of a skeleton multivector of k RHS: value (node, r) at node * ns +
// r * rs.  ns = 0 stands for node-major [N_s][k] (ns = k, rs = 1); RHS-major
// [k][N_s] is ns = 1, rs = N_s.
struct SkelStride {
    uint32_t ns = 0;
    int64_t rs = 0;
};
inline SkelStride skel_stride(SkelStride s, int k) {
    if (s.ns == 0) return SkelStride{(uint32_t)k, 1};
    return s;
}

// Per-RHS scalars of the conjugate gradients (device arrays of k entries).
struct CgState {
    double* rho;     // r.z
    double* pq;      // p.q
    double* alpha;
    double* beta;
    double* rr;      // r.r
    double* bb;      // b.b
    double* tol2;    // tol^2 (same for all RHS)
    int* active;     // 1 while iterating
    int* iters;
    int* status;
    // Stagnation exit (window > 0, inner solves of the refinement): rrb holds
    // r.r at the last time the residual norm halved, stall the iterations since.
    double* rrb;
    int* stall;
    int window;
    // Nullable, [k]: added to r.z in RED_INIT / RED_RZ (the coarse part
    // r0 . A_0^-1 r0 of the two-level preconditioner)
    const double* rz_extra = nullptr;
    // [k]: the step length whose x update a deferring step left pending (its
    // direction is still in p), 0 if none; set by RED_INIT* and RED_RZ*
    double* xa = nullptr;
};

// Per-iteration view of the CG state for kernels that complete a reduction of
// their producer themselves (every workgroup reduces the partial sums in one
// fixed order, so all take identical decisions; one workgroup per RHS stores
// the state).  rho and active have two slots that alternate with the
// iteration's parity: *_prev is the previous iteration's, rho / act this one's,
// so no kernel reads a slot that it writes.
struct CgFuse {
    const double* part;    // apply: previous step's partials [2][nsb][k] (r.z, r.r); null: none
    int nsb;
    const double* energy;  // step: element energies [n_e][k] of this iteration's apply
    int64_t n_e;
    const double* rho_prev;
    const int* act_prev;
    double* rho;
    int* act;
    double* beta;
    double* rr;
    int* iters;
    int* status;
    const double* bb;
    const double* tol2;
    double* pq;
    // alpha has two slots too: the step stores this iteration's into alpha and
    // reads the previous iteration's from alpha_prev (x_mode CG_X_FLUSH)
    double* alpha;
    const double* alpha_prev;
    int x_mode;  // the step's CgXMode
    // stagnation state with the same two slots as rho (see CgState)
    const double* rrb_prev;
    double* rrb;
    const int* stall_prev;
    int* stall;
    int window;
    int* host_act;  // nullable: pinned host copy of act as epoch2 + act, written with it
    int epoch2;     // twice the number of the solve call (flags of earlier calls never match)
};

template <typename T>
struct ApplyArgs {
    Geo g;
    DevTab<T> tab;
    const T* u;       // k skeleton vectors, transformed basis: value (node, r) at node*ns + r*rs
    T* v;             // same layout, accumulated into (zero it first)
    int k;
    uint32_t ns = 0;  // node stride: k for [N_s][k] (RHS innermost), 1 for [k][N_s]
    uint32_t rs = 0;  // RHS stride: 1 for [N_s][k], N_s for [k][N_s]
    int read_con = 0; // 1: read entities on Dirichlet faces too (lifting of prescribed values);
                      //    their outputs are never written either way
    double* energy;   // nullable, [n_elem][k]: element energies u_e . (H~^ u)_e
    int64_t e_begin;  // first element of this launch
    // Fused CG direction (all null for a plain apply): when dir_r is set the
    // operand is p = beta_r u + pinv r, formed at the gather with fmadd, where
    // u holds the previous direction and beta the per-RHS coefficients [k].
    // Such applies take RHS-major vectors (ns = 1) and address them, and the
    // slots, with 32-bit byte offsets (N_s and qlen times sizeof(T) < 2^32).
    const T* dir_r = nullptr;
    const T* dir_pinv = nullptr;
    const double* dir_beta = nullptr;
    // With DIR and fz.part set, beta is not read from dir_beta: every
    // workgroup completes the previous step's r.z reduction itself (RED_RZ),
    // and the workgroups of x = 0 store the new state.
    CgFuse fz = {};
    // Nullable, [k]: right-hand sides r with act[r] == 0 are skipped (stopped CG
    // right-hand sides in the loop with separate reductions).
    const int* act = nullptr;
    // Nullable: the element rows of edges and vertices (and of faces when
    // face_slots) are stored into per-side slots (layout.h)
    // slots[r * qlen + slot_addr(node, slot)] instead of being added into v
    // (RHS-major only, ns = 1).  Face rows otherwise go into v: two additions
    // into zero, whose result does not depend on their order.
    T* slots = nullptr;
    int64_t qlen = 0;
    int face_slots = 0;
    // Nullable (FP32, 6 <= n_I <= 15): D^-1 of the fast diagonalisation per
    // metric class, [class][n_I^3] in (k, j, i) order, and the class of every
    // element; without it D^-1 is recomputed at every eigenspace point.
    const T* dinv = nullptr;
    const int* dcls = nullptr;
};

constexpr int kMaxRhs = 256;  // right-hand sides per call

template <typename T>
hipError_t launch_apply_tpt(const ApplyArgs<T>& a, int64_t n_elem, hipStream_t st);

// D^-1 tables of nc metric classes (dclass: [nc][4] coefficients d_0..d_3):
// out = 1 / (d_0 + d_1 Lambda_i + d_2 Lambda_j + d_3 Lambda_k), evaluated in
// FP64 and rounded once to FP32, [nc][NI][NI][NI] in (k, j, i) order.
hipError_t launch_dinv_table(const double* lam, int NI, const double* dclass, int nc, float* out, hipStream_t st);

// Basis change of skeleton arrays: per face out = A in A^T over the face's two
// interior axes, per edge out = A in, vertices copied.  A is n_I x n_I row-major.
template <typename T>
hipError_t launch_transform(const Layout& L, const T* A, const T* in, T* out, int k, hipStream_t st,
                            SkelStride sk = {});

// Assembly R from per-side slots (layout.h), RHS-major [k][qlen]: out(node, r)
// at node * ns + r * rs, every node written.
template <typename T>
hipError_t launch_slot_sum(const Layout& L, const T* slots, int64_t qlen, T* out, int k, uint32_t ns, uint32_t rs,
                           hipStream_t st);

// diag(R H~^_L R^T) into diag (FP64).  slots (nullable, slot_len doubles,
// zeroed): element rows go to per-side slots summed in a fixed order, so the
// result does not depend on scheduling; without, diag (zeroed first)
// accumulates them with atomics.
hipError_t launch_precond_diag(const Geo& g, const DevTab<double>& tab, double* diag, double* slots, hipStream_t st);
// pinv[s] = 1/diag[s] on free slots, 0 on constrained ones (type T).
template <typename T>
hipError_t launch_precond_invert(const Layout& L, const double* diag, T* pinv, hipStream_t st);

// Condensed transformed RHS, accumulated into fhat (zeroed first).  The element
// cube of (p+1)^3 values lives in LDS when it fits, else in `scratch`
// (grid x (p+1)^3 doubles, grid = number of workgroups used).
// slots (nullable, k * slot_len doubles, zeroed): rows stored per side and
// summed in a fixed order into fhat (every entry written); else fhat (zeroed
// first) accumulates them with atomics.
// rhs_batch: right-hand sides per workgroup of the batched kernels
// (rhs_batched.hip, 8 <= n_I <= 12); 0 keeps one workgroup per (element,
// right-hand side) with the per-item kernels.
hipError_t launch_condense_rhs(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                               double* fhat, int k, double* scratch, int grid, double* slots, hipStream_t st,
                               SkelStride sk = {}, int rhs_batch = 0);
hipError_t launch_condense_rhs_body(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                    double* fhat, int k, double* scratch, int grid, double* slots, int64_t qlen,
                                    hipStream_t st, SkelStride sk = {}, int rhs_batch = 0);
int rhs_grid_for_scratch(int p, int64_t n_e, bool* needs_scratch);

// Interior recovery (Algorithm 4, second loop): u_I = (S(x)S(x)S) D^-1 (F~_I - H~_IB u~_B),
// written into the interior nodes of the nodal array u [k][N].
// keep_con: faces on Dirichlet planes contribute their values in xskel (prescribed
// boundary values) instead of 0.
hipError_t launch_recover_interior(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                   const double* xskel, double* u, int k, double* scratch, int grid,
                                   int keep_con, hipStream_t st, SkelStride sk = {}, int rhs_batch = 0);

// The batched kernels (R right-hand sides per workgroup), for the layouts
// rhs_batched_supported accepts.
bool rhs_batched_supported(const Layout& L, int64_t N);
hipError_t launch_condense_rhs_mb(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                  double* fhat, int k, int R, double* slots, int64_t qlen, hipStream_t st,
                                  SkelStride sk);
hipError_t launch_recover_interior_mb(const Geo& g, const DevTab<double>& tab, const double* f, int64_t N,
                                      const double* xskel, double* u, int k, int R, int keep_con, hipStream_t st,
                                      SkelStride sk);

// Operator variants of Sec. 7 (variants.hip), FP64, physical basis, skeleton
// vectors [N_s][k]: TPC (Algorithm 3 with the suboperators of Table 1; v is
// accumulated into, zero it first) and the gather / scatter around the MMC
// class GEMMs (UL, VL column-major n_B x n_e k, column col_of[e] * k + r).
size_t tpc_smem_bytes(int p);
hipError_t launch_apply_tpc(const Geo& g, const DevTab<double>& tab, const double* K, const double* u, double* v,
                            int k, hipStream_t st);
hipError_t launch_elem_metrics(const Geo& g, double* d, hipStream_t st);

// Two-level preconditioner (coarse.hip): vertex coarse space.  tw = [t_0; t_1]
// (2 n_I doubles), vmap: vertex -> coarse unknown or -1, r0 [k][n0].
template <typename T>
hipError_t launch_coarse_restrict(const Layout& L, const double* tw, const int* vmap, int n0, const T* r, int k,
                                  const int* act, double* r0, hipStream_t st);
hipError_t launch_coarse_dot(const double* a, const double* b, int n0, int k, double* out, hipStream_t st);
hipError_t launch_symmetrize_lower(double* A, int n, hipStream_t st);
// z0 += Ainv r0 (symmetric Ainv, n0 x n0 column-major; r0, z0 [k][n0])
hipError_t launch_coarse_gemv(const double* Ainv, int n0, const double* r0, int k, double* z0, hipStream_t st);
template <typename T>
hipError_t launch_coarse_pupd(const Layout& L, const double* tw, const int* vmap, int n0, const double* z0,
                              const T* pinv, const T* r, T* p, int k, CgState s, hipStream_t st);
hipError_t launch_mmc_gather(const Layout& L, const int* col_of, const double* u, double* UL, int k, hipStream_t st);
hipError_t launch_mmc_scatter(const Layout& L, const int* col_of, const double* VL, double* v, int k, hipStream_t st);

// Skeleton <-> nodal copies (FP64).
// keep_con: copy the values of Dirichlet nodes too (else they are written as 0).
hipError_t launch_skel_to_nodal(const Layout& L, const double* skel, double* nodal, int64_t N, int k,
                                int keep_con, hipStream_t st, SkelStride sk = {});
// Zero the entries of free nodes (keep = constrained) or of Dirichlet nodes
// (keep = free) of an [N_s][k] array.
enum KeepNodes { KEEP_FREE = 0, KEEP_CONSTRAINED = 1 };
hipError_t launch_mask_nodes(const Layout& L, double* x, int k, int keep, hipStream_t st);
// y += a x (n values).
hipError_t launch_axpy(double* y, const double* x, double a, int64_t n, hipStream_t st);
hipError_t launch_nodal_to_skel(const Layout& L, const double* nodal, double* skel, int64_t N, int k,
                                hipStream_t st);

// Assembled GLL-lumped nodal mass M_G [N] (w: p+1 GLL weights on the device).
hipError_t launch_nodal_mass(const Geo& g, const double* w, double* mass, int64_t N, hipStream_t st);
// out = in * M_G (or in / M_G when inverse), nodal [k][N].
hipError_t launch_mass_apply(const Geo& g, const double* w, const double* in, double* out, int64_t N, int k,
                             int inverse, hipStream_t st);
// grad[e][m] = -sum_r a_e^T A_m u_e (m = 0..3), grad[e][4] = J_e grad[e][0]  ([n_e][5]);
// per_rhs: grad[e][m][r] = -a_{e,r}^T A_m u_{e,r}  ([n_e][4][k]).
hipError_t launch_element_grads(const Geo& g, const double* w, const double* K, const double* u, const double* a,
                                int64_t N, int k, double* grad, bool per_rhs, hipStream_t st);

template <typename T>
hipError_t launch_fill(T* x, int64_t n, T val, hipStream_t st);
template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* in, Tout* out, int64_t n, hipStream_t st);
// out = active[r] ? float(in) : 0 per right-hand side r of a [k][n/k] array.
hipError_t launch_convert_masked(const double* in, float* out, int64_t n, int k, const int* active, hipStream_t st);
// x += double(d).
hipError_t launch_add_mixed(double* x, const float* d, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// Conjugate gradients (BT solver, Sec. 8) on RHS-major multivectors [k][N_s]
// (each right-hand side contiguous, so the apply's per-RHS gathers and
// scatters are as coalesced as for one RHS).  Device state holds per-RHS
// scalars; reductions are two-stage and in a fixed order, so results do not
// depend on scheduling.
// ---------------------------------------------------------------------------

constexpr int kVecBlocks = 2048;  // vector-kernel blocks over all RHS

// Blocks per RHS of the vector kernels (the partials per RHS): kVecBlocks / k.
int vec_blocks(int k);

// out = in^T for an R x C row-major array ([N_s][k] <-> [k][N_s]).
template <typename T>
hipError_t launch_transpose(const T* in, T* out, int64_t R, int64_t C, hipStream_t st);

// r = b - q0 (q0 nullable: then r = b; else q0 is zeroed after use), p = 0
// (the previous direction of the first step, whose beta is 0) unless keep_p,
// partials[0]: r.z, [1]: r.r, [2]: b.b  ([3][vec_blocks(k)][k] doubles).
template <typename T>
hipError_t launch_cg_init(const T* b, T* q0, const T* pinv, T* r, T* p, int64_t Ns, int k,
                          double* partials, hipStream_t st, bool keep_p = false);
// Reduce [nparts][k] partials of `nq` quantities; mode selects the CG step logic.
// RED_INIT_KEEP is RED_INIT for a CG that continues the direction p left by a
// previous solve (cg_init with keep_p): beta = r.z / rho, rho being the r.z that
// formed that solve's last direction (kept when it converged).  RED_RZ_DEFER
// is RED_RZ after a step that deferred its x update (CG_X_DEFER): the step
// length is kept in xa for the next step or for launch_cg_x_flush.
enum ReduceMode { RED_INIT = 0, RED_PQ = 1, RED_RZ = 2, RED_INIT_KEEP = 3, RED_RZ_DEFER = 4 };
hipError_t launch_cg_reduce(const double* partials, int64_t nparts, int nq, int k, CgState s, int mode,
                            hipStream_t st);
// p.q of every RHS from the element energies [n_e][k] in two fixed-order
// stages (block partials into epart [kEnergyBlocks][k], then k_cg_reduce in
// mode RED_PQ), the same result for every run.
constexpr int kEnergyBlocks = 256;
hipError_t launch_energy_pq(const double* energy, int64_t n_e, int k, double* epart, CgState s, hipStream_t st);
// One CG step on active right-hand sides, with q = H~^ p already formed:
// p = fmadd(beta, p, pinv r) (the direction the apply used), x += alpha p,
// r -= alpha q; then q = 0 and partials[0] r.z (z = pinv r), [1] r.r.  Blocks
// of stopped right-hand sides return at once.  With qs (nullable) q of edge and
// vertex nodes (of all nodes with face_slots) is the slot sum of the apply's
// per-side slots (qs + rhs * qlen, layout.h) and only the q entries that the
// apply added into are cleared.  p_formed: p already holds the direction the
// apply used (it is only read), instead of beta p + P^-1 r being formed here.
// x_mode (with p formed here): CG_X_NOW updates x; CG_X_DEFER leaves x alone
// (x is then read and written every other step: x += xa p_old + alpha p at the
// next, CG_X_FLUSH, step, xa being the deferring step's length).  A solve whose
// last step deferred ends with launch_cg_x_flush.
enum CgXMode { CG_X_NOW = 0, CG_X_DEFER = 1, CG_X_FLUSH = 2 };
template <typename T>
hipError_t launch_cg_step(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, CgState s,
                          double* partials, const T* qs, int64_t qlen, const Layout& L, int face_slots,
                          hipStream_t st, bool p_formed = false, int x_mode = CG_X_NOW);
// x += alpha0 p for the right-hand sides whose step count iters is odd (their
// last step, of even index, deferred its update; alpha0: the even iterations'
// alpha slot): the end of a fused loop.
template <typename T>
hipError_t launch_cg_x_flush_parity(T* x, const T* p, int64_t Ns, int k, const int* iters, const double* alpha0,
                                    hipStream_t st);
// x += s.xa p for the right-hand sides with a pending update (xa != 0), then
// xa = 0: the end of a solve whose steps deferred x updates.
template <typename T>
hipError_t launch_cg_x_flush(T* x, const T* p, int64_t Ns, int k, CgState s, hipStream_t st);
// The same step with p.q completed by every block from the element energies
// f.energy (RED_PQ on slot f.rho / f.act; blocks x = 0 store pq, alpha and a
// breakdown); partials [2][fused_step_blocks(k)][k] of r.z and r.r for the next
// apply's fused completion.  f.x_mode as launch_cg_step's x_mode, with the
// deferring step's length in f.alpha_prev at the flushing step; a loop whose
// even iterations defer ends with launch_cg_x_flush_parity.
constexpr int kFusedStepThreads = 1024;
int fused_step_blocks(int k);
template <typename T>
hipError_t launch_cg_step_fused(T* x, T* r, T* p, T* q, const T* pinv, int64_t Ns, int k, const CgFuse& f,
                                double* partials, const T* qs, int64_t qlen, const Layout& L, int face_slots,
                                hipStream_t st);

}  // namespace semcond
