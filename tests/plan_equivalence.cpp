// The planner's two Partition paths give the same tasks: weights summed in
// closed form (no sample estimate, no class list asked for) and the weight
// arrays walked row by row (a class list asked for).  Random multi-instance
// first-level class sizes, stored widths and projection flags; Partition's
// alpha, the no-split flag and the worker count vary.  Host only: the
// planner touches no device without an estimate.
#include <cstdio>
#include <random>

#include "fim_plan.h"

using namespace fim;

int main() {
    std::mt19937_64 g(7);
    int bad = 0;
    for (int trial = 0; trial < 40; trial++) {
        const uint32_t n_inst = 1 + g() % 24;
        std::vector<std::vector<uint32_t>> l2o(n_inst), l2a(n_inst), sup(n_inst), ior(n_inst), roi(n_inst);
        std::vector<PlanInput> in(n_inst);
        for (uint32_t q = 0; q < n_inst; q++) {
            const uint32_t n = 2 + g() % 1500;
            l2o[q].assign(1, 0);
            for (uint32_t i = 0; i < n; i++) {
                uint32_t f = (g() % 4 == 0) ? g() % (n - i) : g() % 8;
                if (f > n - 1 - i) f = n - 1 - i;
                l2o[q].push_back(l2o[q].back() + f);
            }
            l2a[q].assign(l2o[q].back(), 0);
            sup[q].resize(n);
            for (auto &x : sup[q]) x = 1 + g() % 200000;
            const uint32_t W = 1 + g() % 7000;
            in[q].db = nullptr;
            in[q].minsup = 1;
            in[q].n_freq = n;
            in[q].W = W;
            in[q].item_of_rank = &ior[q];
            in[q].rank_of_item = &roi[q];
            in[q].l2_off = &l2o[q];
            in[q].l2_atom = &l2a[q];
            in[q].supp_of_rank = &sup[q];
            in[q].Wp = (W + 3) / 4 * 4;
            in[q].project = g() % 2;
            in[q].estimate = false;
        }
        fim_options o{};
        o.alpha = (trial % 3 == 0) ? 0.05 : 0.3;
        o.flags = (trial % 7 == 0) ? FIM_FLAG_NO_SPLIT : 0;
        const uint32_t nw = 256 + 256 * (g() % 8);
        std::vector<std::vector<double>> none(n_inst);
        std::vector<Task> a, b;
        std::vector<PlanClass> cls;
        if (plan_tasks(nullptr, in, o, nw, a, &cls, nullptr, nullptr, &none) != FIM_OK ||
            plan_tasks(nullptr, in, o, nw, b, nullptr, nullptr, nullptr, &none) != FIM_OK) {
            printf("trial %d: planner error\n", trial);
            return 2;
        }
        bool same = a.size() == b.size();
        for (size_t k = 0; same && k < a.size(); k++)
            same = a[k].inst == b[k].inst && a[k].node == b[k].node && a[k].r0 == b[k].r0 &&
                   a[k].r1 == b[k].r1;
        if (!same) {
            printf("trial %d: %zu tasks against %zu\n", trial, a.size(), b.size());
            bad++;
        }
    }
    printf("mismatching trials: %d\n", bad);
    return bad != 0;
}
