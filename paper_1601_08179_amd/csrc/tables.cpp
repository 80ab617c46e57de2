// Host 1D tables of the spectral basis and of the fast diagonalisation.
//
// Sec. 3: GLL nodes and weights of degree p, GLL-lumped mass M = diag(w),
// stiffness K_ij = int phi_i' phi_j'.  Sec. 5 (eq. generalized_eigenvalues):
// generalized eigenpairs of (K_II, M_II), taken in the convention
// S^T M_II S = I, S^T K_II S = Lambda.  Sec. 6: the transformed 1D matrices
// M~ = diag(M_00, I, M_pp) and K~ with interior block Lambda and coupling
// columns a = S^T K_I0, b = S^T K_Ip.
//
// Everything is computed in x87 extended precision (long double) and rounded
// once, so that K and the derived vectors are accurate to about one unit in
// the last place of FP64 up to p = 32.

#include "tables.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace semcond {

namespace {

typedef long double ld;

// Legendre P_p and P_p' at x by the three-term recurrence.
void legendre(int p, ld x, ld* P, ld* dP) {
    ld p0 = 1.0L, p1 = x;
    if (p == 0) { *P = 1.0L; *dP = 0.0L; return; }
    for (int m = 1; m < p; ++m) {
        ld p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    // P_p' = p (x P_p - P_{p-1}) / (x^2 - 1), valid away from +-1
    *dP = (ld)p * (x * p1 - p0) / (x * x - 1.0L);
}

// Cyclic Jacobi eigen-solver for a symmetric n x n matrix A (row-major, destroyed).
// On return the diagonal of A holds the eigenvalues and V (row-major) the
// eigenvectors as columns.
void jacobi_eigen(int n, std::vector<ld>& A, std::vector<ld>& V) {
    V.assign((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0L;
    for (int sweep = 0; sweep < 100; ++sweep) {
        ld off = 0.0L, diag = 0.0L;
        for (int i = 0; i < n; ++i) {
            diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
            for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        }
        if (off <= 1e-40L * diag) break;
        for (int pp = 0; pp < n; ++pp) {
            for (int q = pp + 1; q < n; ++q) {
                ld apq = A[(size_t)pp * n + q];
                if (apq == 0.0L) continue;
                ld app = A[(size_t)pp * n + pp], aqq = A[(size_t)q * n + q];
                ld theta = (aqq - app) / (2.0L * apq);
                ld t = (theta >= 0 ? 1.0L : -1.0L) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0L));
                ld c = 1.0L / std::sqrt(t * t + 1.0L), s = t * c;
                for (int r = 0; r < n; ++r) {
                    ld arp = A[(size_t)r * n + pp], arq = A[(size_t)r * n + q];
                    A[(size_t)r * n + pp] = c * arp - s * arq;
                    A[(size_t)r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {
                    ld apr = A[(size_t)pp * n + r], aqr = A[(size_t)q * n + r];
                    A[(size_t)pp * n + r] = c * apr - s * aqr;
                    A[(size_t)q * n + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < n; ++r) {
                    ld vrp = V[(size_t)r * n + pp], vrq = V[(size_t)r * n + q];
                    V[(size_t)r * n + pp] = c * vrp - s * vrq;
                    V[(size_t)r * n + q] = s * vrp + c * vrq;
                }
            }
        }
    }
}

}  // namespace

bool build_tables(int p, Tables1D* t) {
    if (p < 2 || p > kMaxP) return false;
    const int n = p + 1, NI = p - 1;
    t->p = p;
    t->NI = NI;

    // GLL nodes: -1, 1 and the roots of P_p' (Newton from Chebyshev-Lobatto guesses).
    std::vector<ld> x(n), w(n), Pn(n);
    for (int i = 0; i < n; ++i) x[i] = -std::cos((ld)M_PI * i / p);
    for (int i = 1; i < p; ++i) {
        ld xi = x[i];
        for (int it = 0; it < 100; ++it) {
            ld P, dP;
            legendre(p, xi, &P, &dP);
            ld d2P = (2.0L * xi * dP - (ld)p * (p + 1) * P) / (1.0L - xi * xi);
            ld dx = dP / d2P;
            xi -= dx;
            if (std::fabs(dx) < 1e-21L) break;
        }
        x[i] = xi;
    }
    x[0] = -1.0L;
    x[p] = 1.0L;
    for (int i = 0; i < n; ++i) {
        ld P, dP;
        legendre(p, x[i], &P, &dP);
        Pn[i] = P;
        w[i] = 2.0L / ((ld)p * (p + 1) * P * P);
    }
    // Differentiation matrix D_ij = phi_j'(x_i) = P_p(x_i) / (P_p(x_j) (x_i - x_j)),
    // diagonal by the negative row sum.
    std::vector<ld> D((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        ld s = 0.0L;
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            ld v = Pn[i] / (Pn[j] * (x[i] - x[j]));
            D[(size_t)i * n + j] = v;
            s += v;
        }
        D[(size_t)i * n + i] = -s;
    }
    // K = D^T W D (exact GLL quadrature of phi_i' phi_j', degree 2p-2).
    std::vector<ld> K((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            ld s = 0.0L;
            for (int q = 0; q < n; ++q) s += D[(size_t)q * n + i] * w[q] * D[(size_t)q * n + j];
            K[(size_t)i * n + j] = s;
            K[(size_t)j * n + i] = s;
        }

    // Generalized eigenproblem K_II s = lambda M_II s through the symmetric
    // form C = M_II^-1/2 K_II M_II^-1/2 = Q Lambda Q^T, S = M_II^-1/2 Q.
    std::vector<ld> C((size_t)NI * NI), Q;
    for (int i = 0; i < NI; ++i)
        for (int j = 0; j < NI; ++j)
            C[(size_t)i * NI + j] = K[(size_t)(i + 1) * n + (j + 1)] / std::sqrt(w[i + 1] * w[j + 1]);
    jacobi_eigen(NI, C, Q);
    std::vector<int> order(NI);
    for (int i = 0; i < NI; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return C[(size_t)a * NI + a] < C[(size_t)b * NI + b];
    });
    std::vector<ld> S((size_t)NI * NI), lam(NI);
    for (int m = 0; m < NI; ++m) {
        int src = order[m];
        lam[m] = C[(size_t)src * NI + src];
        // sign convention: the first nonzero component of each column positive
        ld sgn = 1.0L;
        for (int i = 0; i < NI; ++i) {
            ld v = Q[(size_t)i * NI + src];
            if (std::fabs(v) > 1e-12L) { sgn = v > 0 ? 1.0L : -1.0L; break; }
        }
        for (int i = 0; i < NI; ++i)
            S[(size_t)i * NI + m] = sgn * Q[(size_t)i * NI + src] / std::sqrt(w[i + 1]);
    }

    t->x.resize(n);
    t->w.resize(n);
    t->K.resize((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        t->x[i] = (double)x[i];
        t->w[i] = (double)w[i];
    }
    for (size_t i = 0; i < K.size(); ++i) t->K[i] = (double)K[i];
    t->S.resize((size_t)NI * NI);
    t->Sinv.resize((size_t)NI * NI);
    t->SinvT.resize((size_t)NI * NI);
    t->lam.resize(NI);
    t->a.resize(NI);
    t->b.resize(NI);
    for (int i = 0; i < NI; ++i)
        for (int m = 0; m < NI; ++m) {
            t->S[(size_t)i * NI + m] = (double)S[(size_t)i * NI + m];
            // S^-1 = S^T M_II:  (S^-1)_{m i} = S_{i m} w_i
            t->Sinv[(size_t)m * NI + i] = (double)(S[(size_t)i * NI + m] * w[i + 1]);
            // S^-T = M_II S:    (S^-T)_{i m} = w_i S_{i m}
            t->SinvT[(size_t)i * NI + m] = (double)(w[i + 1] * S[(size_t)i * NI + m]);
        }
    for (int m = 0; m < NI; ++m) {
        t->lam[m] = (double)lam[m];
        ld am = 0.0L, bm = 0.0L;
        for (int i = 0; i < NI; ++i) {
            am += S[(size_t)i * NI + m] * K[(size_t)(i + 1) * n + 0];
            bm += S[(size_t)i * NI + m] * K[(size_t)(i + 1) * n + p];
        }
        t->a[m] = (double)am;
        t->b[m] = (double)bm;
    }
    t->m0 = (double)w[0];
    t->K00 = (double)K[0];
    t->K0p = (double)K[p];
    return true;
}

}  // namespace semcond
