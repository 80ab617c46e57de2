// Structured skeleton layout: entity-major, right-hand side innermost.
//
// The skeleton (element faces, edges, vertices; Sec. 4 boundary set B) is
// stored as seven arrays laid end to end, each entity's nodes contiguous:
//   Fx[n3][n2][n1+1][k_I][j_I]  faces normal to x1 (w/e of the elements)
//   Fy[n3][n2+1][n1][k_I][i_I]  faces normal to x2 (s/n)
//   Fz[n3+1][n2][n1][j_I][i_I]  faces normal to x3 (b/t)
//   Ex[n3+1][n2+1][n1][i_I]     edges along x1
//   Ey[n3+1][n2][n1+1][j_I]     edges along x2
//   Ez[n3][n2+1][n1+1][k_I]     edges along x3
//   V [n3+1][n2+1][n1+1]        vertices
// with i_I, j_I, k_I = 0..n_I-1 the interior GLL index (local index minus 1).
// A node index s addresses the values s*k + r, r = 0..k-1.
//
// Gather R^T and scatter R of Sec. 3 reduce to this index arithmetic: element
// (e1,e2,e3) reads w = Fx[e3][e2][e1], e = Fx[e3][e2][e1+1], s = Fy[e3][e2][e1],
// n = Fy[e3][e2+1][e1], b = Fz[e3][e2][e1], t = Fz[e3+1][e2][e1]; edge X(jb,kb) =
// Ex[e3+kb][e2+jb][e1], Y(ib,kb) = Ey[e3+kb][e2][e1+ib], Z(ib,jb) =
// Ez[e3][e2+jb][e1+ib]; vertex (ib,jb,kb) = V[e3+kb][e2+jb][e1+ib].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace semcond {

struct Layout {
    int n1, n2, n3, NI, p;
    unsigned mask;  // Dirichlet bits: 0 x1-low, 1 x1-high, 2 x2-low, 3 x2-high, 4 x3-low, 5 x3-high
    int64_t oFx, oFy, oFz, oEx, oEy, oEz, oV, Ns;
};

inline Layout make_layout(int p, const int n[3], unsigned mask) {
    Layout L;
    L.n1 = n[0];
    L.n2 = n[1];
    L.n3 = n[2];
    L.p = p;
    L.NI = p - 1;
    L.mask = mask;
    const int64_t n1 = n[0], n2 = n[1], n3 = n[2], NI = p - 1, NI2 = NI * NI;
    L.oFx = 0;
    L.oFy = L.oFx + n3 * n2 * (n1 + 1) * NI2;
    L.oFz = L.oFy + n3 * (n2 + 1) * n1 * NI2;
    L.oEx = L.oFz + (n3 + 1) * n2 * n1 * NI2;
    L.oEy = L.oEx + (n3 + 1) * (n2 + 1) * n1 * NI;
    L.oEz = L.oEy + (n3 + 1) * n2 * (n1 + 1) * NI;
    L.oV = L.oEz + n3 * (n2 + 1) * (n1 + 1) * NI;
    L.Ns = L.oV + (n3 + 1) * (n2 + 1) * (n1 + 1);
    return L;
}

// Entity base node indices.
__host__ __device__ inline int64_t fx_base(const Layout& L, int e3, int e2, int fx) {
    return L.oFx + (((int64_t)e3 * L.n2 + e2) * (L.n1 + 1) + fx) * L.NI * L.NI;
}
__host__ __device__ inline int64_t fy_base(const Layout& L, int e3, int fy, int e1) {
    return L.oFy + (((int64_t)e3 * (L.n2 + 1) + fy) * L.n1 + e1) * L.NI * L.NI;
}
__host__ __device__ inline int64_t fz_base(const Layout& L, int fz, int e2, int e1) {
    return L.oFz + (((int64_t)fz * L.n2 + e2) * L.n1 + e1) * L.NI * L.NI;
}
__host__ __device__ inline int64_t ex_base(const Layout& L, int ez, int ey, int e1) {
    return L.oEx + (((int64_t)ez * (L.n2 + 1) + ey) * L.n1 + e1) * L.NI;
}
__host__ __device__ inline int64_t ey_base(const Layout& L, int ez, int e2, int ex) {
    return L.oEy + (((int64_t)ez * L.n2 + e2) * (L.n1 + 1) + ex) * L.NI;
}
__host__ __device__ inline int64_t ez_base(const Layout& L, int e3, int ey, int ex) {
    return L.oEz + (((int64_t)e3 * (L.n2 + 1) + ey) * (L.n1 + 1) + ex) * L.NI;
}
__host__ __device__ inline int64_t v_base(const Layout& L, int vz, int vy, int vx) {
    return L.oV + ((int64_t)vz * (L.n2 + 1) + vy) * (L.n1 + 1) + vx;
}

// Per-side output slots of the condensed operator inside the conjugate
// gradients: every element stores its rows of a shared entity into a slot of
// its own (plain stores), and the assembly R becomes a fixed-order sum of the
// slots of a node.  A face node has 2 slots (slot 1 - side of the element's
// face: w, s, b -> 1; e, n, t -> 0), an edge node 4 ((1 - b0) + 2 (1 - b1) for
// the element's boundary bits of the edge), a vertex 8 ((1 - ib) + 2 (1 - jb) +
// 4 (1 - kb)).  Per right-hand side: [2][N_s] (slots 0 and 1 of every node),
// [2][edge nodes] (slots 2, 3 of edges), [6][vertices] (slots 2..7).  Slots
// that no element writes (domain boundary sides, Dirichlet entities) hold 0.
__host__ __device__ inline int64_t slot_len(const Layout& L) {
    return 2 * L.Ns + 2 * (L.oV - L.oEx) + 6 * (L.Ns - L.oV);
}
// Offset of (node, slot) within one right-hand side (slot_len < 2^31).
__host__ __device__ inline uint32_t slot_addr(const Layout& L, uint32_t node, int slot) {
    const uint32_t Ns = (uint32_t)L.Ns, oEx = (uint32_t)L.oEx, oV = (uint32_t)L.oV;
    // (selects instead of lane-by-uniform products where the slot is a bit)
    if (slot < 2) return (slot ? Ns : 0u) + node;
    const uint32_t nE = oV - oEx;
    if (node < oV) return 2 * Ns + (slot == 3 ? nE : 0u) + (node - oEx);
    return 2 * Ns + 2 * nE + (uint32_t)(slot - 2) * (Ns - oV) + (node - oV);
}
// Slot of element entity `id` (the numbering of element_entity below) for the
// element's side of that entity.
__host__ __device__ inline int entity_slot(int id) {
    if (id < 6) return 1 - (id & 1);
    if (id < 18) {
        const int q = (id - 6) & 3;
        return (1 - (q & 1)) + 2 * (1 - (q >> 1));
    }
    const int q = id - 18;
    return (1 - (q & 1)) + 2 * (1 - ((q >> 1) & 1)) + 4 * (1 - (q >> 2));
}
// Assembled value of a node: its slots summed in slot order (faces: only with
// face slots; otherwise a face node's value is the atomic sum in q).
template <typename T>
__host__ __device__ inline T slot_sum(const Layout& L, const T* Q, uint32_t node) {
    const uint32_t Ns = (uint32_t)L.Ns, oEx = (uint32_t)L.oEx, oV = (uint32_t)L.oV;
    T v = Q[node] + Q[Ns + node];
    if (node >= oEx) {
        const uint32_t nE = oV - oEx;
        if (node < oV) {
            const uint32_t b = 2 * Ns + (node - oEx);
            v += Q[b];
            v += Q[b + nE];
        } else {
            const uint32_t nV = Ns - oV, b = 2 * Ns + 2 * nE + (node - oV);
            for (int s = 0; s < 6; ++s) v += Q[b + (uint32_t)s * nV];
        }
    }
    return v;
}

// Is a grid plane on a Dirichlet domain face?
__host__ __device__ inline bool xcon(const Layout& L, int x) {
    return (x == 0 && (L.mask & 1u)) || (x == L.n1 && (L.mask & 2u));
}
__host__ __device__ inline bool ycon(const Layout& L, int y) {
    return (y == 0 && (L.mask & 4u)) || (y == L.n2 && (L.mask & 8u));
}
__host__ __device__ inline bool zcon(const Layout& L, int z) {
    return (z == 0 && (L.mask & 16u)) || (z == L.n3 && (L.mask & 32u));
}

// The 26 skeleton entities of element (e1,e2,e3), in the element's order:
//   0..5   faces w, e, s, n, b, t
//   6..9   edges X(jb,kb) along x1, index jb + 2 kb
//   10..13 edges Y(ib,kb) along x2, index ib + 2 kb
//   14..17 edges Z(ib,jb) along x3, index ib + 2 jb
//   18..25 vertices, index ib + 2 jb + 4 kb
// base[] receives node indices, con[] whether the entity is constrained.
__host__ __device__ inline void element_entity(const Layout& L, int e1, int e2, int e3, int id,
                                               int64_t* base, bool* con) {
    if (id < 6) {
        int side = id & 1;
        if (id < 2) {
            *base = fx_base(L, e3, e2, e1 + side);
            *con = xcon(L, e1 + side);
        } else if (id < 4) {
            *base = fy_base(L, e3, e2 + side, e1);
            *con = ycon(L, e2 + side);
        } else {
            *base = fz_base(L, e3 + side, e2, e1);
            *con = zcon(L, e3 + side);
        }
    } else if (id < 10) {
        int q = id - 6, jb = q & 1, kb = q >> 1;
        *base = ex_base(L, e3 + kb, e2 + jb, e1);
        *con = ycon(L, e2 + jb) || zcon(L, e3 + kb);
    } else if (id < 14) {
        int q = id - 10, ib = q & 1, kb = q >> 1;
        *base = ey_base(L, e3 + kb, e2, e1 + ib);
        *con = xcon(L, e1 + ib) || zcon(L, e3 + kb);
    } else if (id < 18) {
        int q = id - 14, ib = q & 1, jb = q >> 1;
        *base = ez_base(L, e3, e2 + jb, e1 + ib);
        *con = xcon(L, e1 + ib) || ycon(L, e2 + jb);
    } else {
        int q = id - 18, ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
        *base = v_base(L, e3 + kb, e2 + jb, e1 + ib);
        *con = xcon(L, e1 + ib) || ycon(L, e2 + jb) || zcon(L, e3 + kb);
    }
}

// Global GLL indices (I1,I2,I3) of skeleton node s, and whether it is
// constrained, with index arithmetic in type I (32-bit divisions are several
// times cheaper on the GPU than 64-bit ones).
template <typename I>
__host__ __device__ inline void skeleton_node_t(const Layout& L, I s, int* I1, int* I2, int* I3, bool* con) {
    const int p = L.p, NI = L.NI;
    const I NI2 = (I)NI * NI;
    if (s < (I)L.oFy) {
        I t = s - (I)L.oFx, f = t / NI2, loc = t % NI2;
        int k = (int)(loc / (I)NI), j = (int)(loc % (I)NI);
        int fx = (int)(f % (I)(L.n1 + 1));
        I r = f / (I)(L.n1 + 1);
        int e2 = (int)(r % (I)L.n2), e3 = (int)(r / (I)L.n2);
        *I1 = fx * p; *I2 = e2 * p + 1 + j; *I3 = e3 * p + 1 + k;
        *con = xcon(L, fx);
    } else if (s < (I)L.oFz) {
        I t = s - (I)L.oFy, f = t / NI2, loc = t % NI2;
        int k = (int)(loc / (I)NI), i = (int)(loc % (I)NI);
        int e1 = (int)(f % (I)L.n1);
        I r = f / (I)L.n1;
        int fy = (int)(r % (I)(L.n2 + 1)), e3 = (int)(r / (I)(L.n2 + 1));
        *I1 = e1 * p + 1 + i; *I2 = fy * p; *I3 = e3 * p + 1 + k;
        *con = ycon(L, fy);
    } else if (s < (I)L.oEx) {
        I t = s - (I)L.oFz, f = t / NI2, loc = t % NI2;
        int j = (int)(loc / (I)NI), i = (int)(loc % (I)NI);
        int e1 = (int)(f % (I)L.n1);
        I r = f / (I)L.n1;
        int e2 = (int)(r % (I)L.n2), fz = (int)(r / (I)L.n2);
        *I1 = e1 * p + 1 + i; *I2 = e2 * p + 1 + j; *I3 = fz * p;
        *con = zcon(L, fz);
    } else if (s < (I)L.oEy) {
        I t = s - (I)L.oEx, f = t / (I)NI;
        int i = (int)(t % (I)NI);
        int e1 = (int)(f % (I)L.n1);
        I r = f / (I)L.n1;
        int ey = (int)(r % (I)(L.n2 + 1)), ez = (int)(r / (I)(L.n2 + 1));
        *I1 = e1 * p + 1 + i; *I2 = ey * p; *I3 = ez * p;
        *con = ycon(L, ey) || zcon(L, ez);
    } else if (s < (I)L.oEz) {
        I t = s - (I)L.oEy, f = t / (I)NI;
        int j = (int)(t % (I)NI);
        int ex = (int)(f % (I)(L.n1 + 1));
        I r = f / (I)(L.n1 + 1);
        int e2 = (int)(r % (I)L.n2), ez = (int)(r / (I)L.n2);
        *I1 = ex * p; *I2 = e2 * p + 1 + j; *I3 = ez * p;
        *con = xcon(L, ex) || zcon(L, ez);
    } else if (s < (I)L.oV) {
        I t = s - (I)L.oEz, f = t / (I)NI;
        int k = (int)(t % (I)NI);
        int ex = (int)(f % (I)(L.n1 + 1));
        I r = f / (I)(L.n1 + 1);
        int ey = (int)(r % (I)(L.n2 + 1)), e3 = (int)(r / (I)(L.n2 + 1));
        *I1 = ex * p; *I2 = ey * p; *I3 = e3 * p + 1 + k;
        *con = xcon(L, ex) || ycon(L, ey);
    } else {
        I t = s - (I)L.oV;
        int vx = (int)(t % (I)(L.n1 + 1));
        I r = t / (I)(L.n1 + 1);
        int vy = (int)(r % (I)(L.n2 + 1)), vz = (int)(r / (I)(L.n2 + 1));
        *I1 = vx * p; *I2 = vy * p; *I3 = vz * p;
        *con = xcon(L, vx) || ycon(L, vy) || zcon(L, vz);
    }
}

// The same for any skeleton index (the nodal<->skeleton copies and the host
// coords table): 32-bit arithmetic whenever the skeleton has fewer than 2^32
// nodes.
__host__ __device__ inline void skeleton_node(const Layout& L, int64_t s, int* I1, int* I2, int* I3,
                                              bool* con) {
    if (L.Ns <= (int64_t)0xFFFFFFFFu)
        skeleton_node_t<uint32_t>(L, (uint32_t)s, I1, I2, I3, con);
    else
        skeleton_node_t<int64_t>(L, s, I1, I2, I3, con);
}

}  // namespace semcond
