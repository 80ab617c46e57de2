// Host 1D tables (see tables.cpp).
#pragma once

#include <vector>

namespace semcond {

constexpr int kMaxP = 32;
constexpr int kMaxNI = kMaxP - 1;

struct Tables1D {
    int p = 0, NI = 0;
    std::vector<double> x, w;        // GLL nodes and weights, p+1
    std::vector<double> K;           // (p+1)^2 row-major
    std::vector<double> S;           // NI x NI, column m = eigenvector m (S^T M_II S = I)
    std::vector<double> Sinv;        // S^-1 = S^T M_II
    std::vector<double> SinvT;       // S^-T = M_II S
    std::vector<double> lam;         // Lambda, ascending
    std::vector<double> a, b;        // a = S^T K_I0, b = S^T K_Ip
    double m0 = 0, K00 = 0, K0p = 0; // M_00 (= M_pp), K_00 (= K_pp), K_0p
};

bool build_tables(int p, Tables1D* t);

}  // namespace semcond
