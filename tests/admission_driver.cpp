// Host-only driver for the request server's micro-batch choice: prints, for
// seeded random queues, the queue and the indices each rule takes.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "admission.hpp"

static void print_case(char rule, const std::vector<int> &ds, const std::vector<int> &order,
                       int max_batch, int max_datasets, const std::vector<size_t> &taken)
{
    printf("%c %zu %d %d :", rule, ds.size(), max_batch, max_datasets);
    for (int k : ds) printf(" %d", k);
    printf(" :");
    for (int n : order) printf(" %d", n);
    printf(" :");
    for (size_t q : taken) printf(" %zu", q);
    printf("\n");
}

int main(int argc, char **argv)
{
    const int seed = argc > 1 ? atoi(argv[1]) : 1;
    std::mt19937_64 rng(seed);
    for (int c = 0; c < 400; ++c) {
        const size_t queued = rng() % 301;
        const int K = 1 + (int)(rng() % 70);
        const int hot = (int)(rng() % K);   // one frequent dataset
        std::vector<int> ds(queued);
        for (auto &k : ds) k = (rng() % 3 == 0) ? hot : (int)(rng() % K);
        // dataset orders: multiples of 64 up to 6144, with repeats (ties)
        std::vector<int> order(K);
        for (auto &n : order) n = 64 * (1 + (int)(rng() % 96));
        const int max_batch = (int)(rng() % 131);
        const int max_datasets = (int)(rng() % 11);
        auto of = [&](size_t q) { return ds[q]; };
        auto n_of = [&](int k) { return order[k]; };
        print_case('D', ds, order, max_batch, 0, gpk::choose_dataset_batch(queued, of, max_batch));
        print_case('R', ds, order, max_batch, max_datasets,
                   gpk::choose_ragged_batch(queued, of, n_of, max_batch, max_datasets));
    }
    return 0;
}
