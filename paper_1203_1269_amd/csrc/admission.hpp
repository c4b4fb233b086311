// Which queued requests of the request server form its next micro-batch.
// Host logic only (no HIP), so that it is testable on the host.  The queue is
// in arrival order, index 0 the oldest; dataset_of(q) is the dataset of queued
// request q.  Both rules always take the oldest request, so a request waits
// for no more micro-batches than there are older requests.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <vector>

namespace gpk {

// Per-dataset micro-batch: the oldest request's dataset, up to max_batch of
// its queued requests in arrival order.  Returns their queue indices,
// ascending.
template <class DatasetOf>
std::vector<size_t> choose_dataset_batch(size_t queued, const DatasetOf &dataset_of,
                                         int max_batch)
{
    std::vector<size_t> taken;
    if (queued == 0 || max_batch <= 0) return taken;
    const int k = dataset_of(0);
    for (size_t q = 0; q < queued && (int)taken.size() < max_batch; ++q)
        if (dataset_of(q) == k) taken.push_back(q);
    return taken;
}

// Ragged micro-batch: the oldest request's dataset, then the datasets of the
// other queued requests closest to it in order (order_of(k) for dataset k;
// ties go to the dataset whose oldest queued request came first), at most
// max_datasets in all; their queued requests in arrival order, up to
// max_batch.  Matrices of close orders finish their factorisations close
// together, so few panel steps run with only a handful of large matrices
// left.  Returns queue indices, ascending.
template <class DatasetOf, class OrderOf>
std::vector<size_t> choose_ragged_batch(size_t queued, const DatasetOf &dataset_of,
                                        const OrderOf &order_of, int max_batch,
                                        int max_datasets)
{
    std::vector<size_t> taken;
    if (queued == 0 || max_batch <= 0 || max_datasets <= 0) return taken;
    std::vector<int> cand;   // datasets in order of their oldest queued request
    for (size_t q = 0; q < queued; ++q) {
        const int k = dataset_of(q);
        if (std::find(cand.begin(), cand.end(), k) == cand.end()) cand.push_back(k);
    }
    const long n0 = order_of(cand[0]);
    auto dist = [&](int k) {
        const long dn = (long)order_of(k) - n0;
        return dn < 0 ? -dn : dn;
    };
    std::stable_sort(cand.begin() + 1, cand.end(),
                     [&](int a, int b) { return dist(a) < dist(b); });
    if ((int)cand.size() > max_datasets) cand.resize((size_t)max_datasets);
    for (size_t q = 0; q < queued && (int)taken.size() < max_batch; ++q)
        if (std::find(cand.begin(), cand.end(), dataset_of(q)) != cand.end()) taken.push_back(q);
    return taken;
}

}  // namespace gpk
