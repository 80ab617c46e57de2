// Host check of the per-side output slots of the CG applies (layout.h): on
// small meshes with several degrees and Dirichlet masks, every (element,
// entity node) row goes to a distinct in-range slot, and the slot sum of every
// skeleton node reads exactly the slots its elements write.  Exit status 0 on
// success.
#include <cstdio>
#include <set>
#include <vector>

#include "layout.h"

using namespace semcond;

int main() {
    int fails = 0;
    for (int p : {2, 3, 5, 8, 17})
        for (int n1 : {1, 2, 3})
            for (int n2 : {1, 3})
                for (int n3 : {1, 2})
                    for (unsigned mask : {0u, 63u, 5u}) {
                        const int n[3] = {n1, n2, n3};
                        const Layout L = make_layout(p, n, mask);
                        const int NI = p - 1;
                        const int64_t len = slot_len(L);
                        std::vector<int> count(len, 0);
                        std::vector<std::set<uint32_t>> written(L.Ns);
                        for (int e3 = 0; e3 < n3; ++e3)
                            for (int e2 = 0; e2 < n2; ++e2)
                                for (int e1 = 0; e1 < n1; ++e1)
                                    for (int id = 0; id < 26; ++id) {
                                        int64_t base;
                                        bool con;
                                        element_entity(L, e1, e2, e3, id, &base, &con);
                                        int nodes, slot;
                                        if (id < 6) {  // faces w e s n b t: slot 1 - side
                                            nodes = NI * NI;
                                            slot = 1 - (id & 1);
                                        } else if (id < 18) {  // edges: boundary bits (b0, b1)
                                            const int q = (id - 6) % 4, b0 = q & 1, b1 = q >> 1;
                                            nodes = NI;
                                            slot = (1 - b0) + 2 * (1 - b1);
                                        } else {  // vertices (ib, jb, kb)
                                            const int q = id - 18, ib = q & 1, jb = (q >> 1) & 1, kb = q >> 2;
                                            nodes = 1;
                                            slot = (1 - ib) + 2 * (1 - jb) + 4 * (1 - kb);
                                        }
                                        if (con) continue;
                                        for (int l = 0; l < nodes; ++l) {
                                            const uint32_t node = (uint32_t)(base + l);
                                            const uint32_t a = slot_addr(L, node, slot);
                                            if ((int64_t)a >= len) {
                                                std::printf("slot out of range: p %d node %u\n", p, node);
                                                ++fails;
                                                continue;
                                            }
                                            ++count[a];
                                            written[node].insert(a);
                                        }
                                    }
                        for (int64_t a = 0; a < len; ++a)
                            if (count[a] > 1) {
                                std::printf("two rows in one slot: p %d slot %lld\n", p, (long long)a);
                                ++fails;
                                break;
                            }
                        std::vector<double> Q(len, 0.0);
                        for (uint32_t node = 0; node < (uint32_t)L.Ns; ++node) {
                            for (uint32_t a : written[node]) Q[a] = 1.0;
                            const double s = slot_sum(L, Q.data(), node);
                            for (uint32_t a : written[node]) Q[a] = 0.0;
                            if (s != (double)written[node].size()) {
                                std::printf("slot sum of node %u (p %d) reads %g of %zu rows\n", node, p, s,
                                            written[node].size());
                                ++fails;
                                break;
                            }
                        }
                    }
    std::printf("slot layout check: %d failures\n", fails);
    return fails != 0;
}
