// Host model of the persistent product launch's control protocol, one
// std::thread per workgroup, with the kernel's steps in its order:
//  * per product, take tiles from the own XCD's queue through an atomic
//    head, then steal from the other seven queues;
//  * one grid barrier per product: an atomic arrival, then a poll until
//    the arrivals reach (products so far) x (workgroups), bounded by a
//    deadline that raises a shared fail flag;
//  * after the barrier every workgroup reduces the same per-product
//    partials in the same order and takes the same stop decision; only
//    workgroup 0 writes the run state.
// Checks: every tile of every product is taken exactly once, every
// workgroup leaves, all leave at the same product, and no deadline expires.
// Sequentially consistent atomics: the model covers the protocol, not the
// GPU's memory model.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

int main(int argc, char **argv) {
    const int G = argc > 1 ? std::atoi(argv[1]) : 48;          // workgroups
    const int list_len = argc > 2 ? std::atoi(argv[2]) : 6;    // tiles per XCD list (48 tiles / 8)
    const int n_steps = argc > 3 ? std::atoi(argv[3]) : 30;    // product budget
    const int stop_at = argc > 4 ? std::atoi(argv[4]) : 27;    // product at which the stop rule fires
    const unsigned seed = argc > 5 ? (unsigned)std::atoi(argv[5]) : 1u;
    constexpr int kXcds = 8;
    std::atomic<unsigned> arrive{0}, fail{0};
    std::vector<std::atomic<unsigned>> head((size_t)n_steps * kXcds);
    std::vector<std::atomic<int>> taken((size_t)n_steps * kXcds * list_len);
    std::vector<double> partial((size_t)2 * kXcds * list_len, 0.0);    // double-buffered by product parity
    std::vector<int> products_done(G, -1), result(G, -1);
    for (auto &h : head) h = 0;
    for (auto &t : taken) t = 0;
    const auto t_end = std::chrono::steady_clock::now() + std::chrono::seconds(20);
    auto wg = [&](int b) {
        std::mt19937 rng(seed * 7919u + (unsigned)b);
        const int my_x = b % kXcds;
        unsigned n_barriers = 0;
        int kq = 0;                                   // product ordinal (state every workgroup keeps alike)
        while (true) {
            for (int probe = 0; probe < kXcds; ++probe) {
                const int x = (my_x + probe) % kXcds;
                while (true) {
                    const unsigned q = head[(size_t)kq * kXcds + x].fetch_add(1u);
                    if ((int)q >= list_len) break;
                    taken[((size_t)kq * kXcds + x) * list_len + q].fetch_add(1);
                    partial[(size_t)(kq & 1) * kXcds * list_len + x * list_len + q] = 1.0 + kq;
                    if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
                }
            }
            ++n_barriers;
            arrive.fetch_add(1u);
            while (arrive.load() < n_barriers * (unsigned)G) {
                if (fail.load() || std::chrono::steady_clock::now() > t_end) { fail = 1; return; }
                std::this_thread::yield();
            }
            double tr = 0.0;                          // the same reduction in every workgroup
            for (int i = 0; i < kXcds * list_len; ++i) tr += partial[(size_t)(kq & 1) * kXcds * list_len + i];
            const bool stop = kq + 1 >= stop_at || kq + 1 >= n_steps;
            if (tr != (1.0 + kq) * kXcds * list_len) { fail = 2; return; }
            ++kq;
            if (stop) break;
        }
        products_done[b] = kq;
        if (b == 0) result[b] = kq;
    };
    std::vector<std::thread> th;
    for (int b = 0; b < G; ++b) th.emplace_back(wg, b);
    for (auto &t : th) t.join();
    if (fail.load()) { std::printf("FAIL: flag %u\n", fail.load()); return 1; }
    const int expect = stop_at < n_steps ? stop_at : n_steps;
    for (int b = 0; b < G; ++b)
        if (products_done[b] != expect) { std::printf("FAIL: workgroup %d left after %d products\n", b, products_done[b]); return 1; }
    for (int kq = 0; kq < expect; ++kq)
        for (int i = 0; i < kXcds * list_len; ++i)
            if (taken[(size_t)kq * kXcds * list_len + i].load() != 1) {
                std::printf("FAIL: product %d tile %d taken %d times\n", kq, i, taken[(size_t)kq * kXcds * list_len + i].load());
                return 1;
            }
    std::printf("OK: %d workgroups, %d tiles per product, %d products, arrivals %u\n", G, kXcds * list_len, expect,
                arrive.load());
    return 0;
}
