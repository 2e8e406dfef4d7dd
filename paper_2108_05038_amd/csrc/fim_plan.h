// Work planning for the persistent kernel: the thesis's sample-based class
// size estimate (Phase 1, reservoir variant), the Partition of large classes
// and the LPT order (Phase 2).
#pragma once

#include <vector>

#include "fim_host.h"

namespace fim {

struct PlanInput {
    const fim_db *db;
    uint32_t minsup;
    uint32_t n_freq;
    uint32_t W;
    const std::vector<uint32_t> *item_of_rank;
    const std::vector<uint32_t> *rank_of_item;
    const std::vector<uint32_t> *l2_off;   // atoms of the first-level classes
    const std::vector<uint32_t> *l2_atom;
    const std::vector<uint32_t> *supp_of_rank = nullptr;  // supports of the frequent items
    uint32_t Wp = 0;                       // words per stored row
    bool project = false;                  // rows are projected on small prefix covers
    bool estimate = true;                  // draw the database sample for this instance
};

// One class handed to the workers with its estimated size.
struct PlanClass {
    uint32_t inst, node, r0, r1;
    double weight;   // estimated work (comparable across instances)
    double proxy;    // size proxy used to order classes the sample does not see
};

// Default sample sizes.
//  |D~| from Toivonen's Chernoff bound (thesis, theorem on estimating a
//       support from a database sample): ceil(ln(2/delta) / (2 eps^2)),
//  |S|  from the hypergeometric Kullback-Leibler bound (theorem on the
//       estimation error of the size of a subset from a reservoir sample):
//       ceil(-ln(delta/2) / D(rho + eps || rho)), natural logarithms.
uint32_t default_sample_tx(double eps, double delta);
uint32_t default_sample_fi(double rho, double eps, double delta);
double bernoulli_kl(double x, double y);

// Phase 1's database sample: nd transactions drawn uniformly with
// replacement (SplitMix64 from `seed`), each reduced to the items frequent in
// the database; CSR into off / items.
void draw_sample(const fim_db *db, const std::vector<uint32_t> &rank_of_item, uint64_t nd,
                 uint64_t seed, std::vector<uint64_t> &off, std::vector<uint32_t> &items);

// Simple reservoir sampling (thesis, the Simple-Reservoir-Sampling
// algorithm): keeps a uniform sample without replacement of size n of a
// stream.  Returns the indices (positions in the stream) that were kept.
std::vector<uint64_t> reservoir_indices(uint64_t stream_len, uint64_t n, uint64_t seed);

// LPT-Schedule (Graham): jobs in decreasing weight, each to the least
// loaded of p workers (lowest index on ties).  Returns the worker of each
// job and the makespan.
double lpt_schedule(const std::vector<double> &w, uint32_t p, std::vector<uint32_t> &worker);

// Partition + LPT order of first-level classes given per-row weights.
void partition_lpt_order(const std::vector<PlanClass> &cls_in,
                         const std::vector<const double *> &rw,
                         const std::vector<const double *> &rp, double alpha, uint32_t n_workers,
                         bool no_split, std::vector<PlanClass> &out);

// The database samples mined and the reservoir's itemsets of every
// instance (Phase 1).  Needs only the instances' databases, minimum
// supports and frequent items, so it can run while the root-class kernel
// of the same instances is still on the GPU.
struct SampleEstimate {
    std::vector<fim_result *> res;  // per sampled instance: reservoir itemsets, stream length
    std::vector<uint32_t> inst;     // instance index of each res
    bool done = false;
    ~SampleEstimate();
};

fim_status sample_phase(fim_ctx *ctx, const std::vector<PlanInput> &in, const fim_options &opts,
                        SampleEstimate &est);

// Builds the task list of all instances in LPT order.  With est (the
// finished Phase 1 of these instances) the sample is not mined again; with
// `given` (per instance, a weight per second-level class, or empty for no
// estimate) no sample is drawn here at all.  *est_out_words receives an
// estimate of the output words of the whole run (0 without a sample
// estimate).
fim_status plan_tasks(fim_ctx *ctx, const std::vector<PlanInput> &in, const fim_options &opts,
                      uint32_t n_workers, std::vector<Task> &tasks,
                      std::vector<PlanClass> *classes = nullptr, uint64_t *est_out_words = nullptr,
                      SampleEstimate *est = nullptr,
                      const std::vector<std::vector<double>> *given = nullptr);

}  // namespace fim
