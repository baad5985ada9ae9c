// CPU check of the persistent kernel's grid barrier (test infrastructure): the algorithm of
// ct_grid_barrier.hpp with one std::thread per workgroup and host atomics. Built by
// tests/test_grid_barrier.py with g++.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "../../paper_1512_04564_amd/csrc/ct_grid_barrier.hpp"

namespace {

struct HostOps {
    int flag = 0;
    void block_sync() {}
    bool leader() { return true; }
    int load(int *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
    int load_acquire(int *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
    void store(int *p, int v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
    void store_release(int *p, int v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
    int fetch_add(int *p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_ACQ_REL); }
    void release() { std::atomic_thread_fence(std::memory_order_release); }
    void acquire() { std::atomic_thread_fence(std::memory_order_acquire); }
    void pause() { std::this_thread::yield(); }
    void set_block_flag(int v) { flag = v; }
    int block_flag() { return flag; }
};

}  // namespace

extern "C" {

// nblocks workgroups run `phases` phases; in phase p each writes its slot of buffer p % 2 and, after the
// barrier, reads every other slot of that buffer. Workgroup `late` (if >= 0) starts late_ms milliseconds
// late. Returns the number of (workgroup, phase) reads that saw a stale value; *error receives the error
// flag, *completed the number of workgroups that finished all phases, *exited the number that returned.
int barrier_run(int nblocks, int phases, unsigned spin_limit, int late, int late_ms, int *error, int *completed,
                int *exited)
{
    int state[4] = {0, 0, 0, 0};
    std::vector<int> buf(2 * (size_t)nblocks, -1);
    std::atomic<int> stale{0}, done{0}, out{0};
    std::vector<std::thread> th;
    for (int b = 0; b < nblocks; ++b)
        th.emplace_back([&, b]() {
            if (b == late) std::this_thread::sleep_for(std::chrono::milliseconds(late_ms));
            HostOps ops;
            bool ok = true;
            for (int p = 0; p < phases && ok; ++p) {
                __atomic_store_n(&buf[(size_t)(p % 2) * nblocks + b], p, __ATOMIC_RELAXED);
                ok = ct::grid_barrier(ops, state, nblocks, spin_limit);
                if (!ok) break;
                for (int o = 0; o < nblocks; ++o)
                    if (__atomic_load_n(&buf[(size_t)(p % 2) * nblocks + o], __ATOMIC_RELAXED) != p) ++stale;
                ok = ct::grid_barrier(ops, state, nblocks, spin_limit);   // nobody overwrites before all read
                if (ok && p == phases - 1) ++done;
            }
            ++out;
        });
    for (auto &t : th) t.join();
    *error = state[3];
    *completed = done.load();
    *exited = out.load();
    return stale.load();
}

}  // extern "C"
