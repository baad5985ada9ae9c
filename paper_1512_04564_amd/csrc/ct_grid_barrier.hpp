// Bounded grid-wide barrier for the persistent batched solve (host + device).
//
// The algorithm is written once over a policy that supplies the memory operations, so that the same code
// runs in the kernel (HIP atomics at agent scope, fences, the workgroup barrier) and in a CPU test (one
// std::thread per workgroup, std::atomic), where its phase ordering and its error path are checked.
//
// State (four ints in device memory, zeroed before the launch): [1] arrivals at the current barrier,
// [2] generation, [3] error flag. A workgroup arrives by publishing its writes (release fence), adding one
// to the arrivals and, unless it is the last, waiting for the generation to change; the last one resets the
// arrivals and advances the generation. Every wait is bounded: after spin_limit polls the waiter raises the
// error flag and leaves, and every workgroup that meets a barrier with the flag raised leaves at once, so
// the kernel always ends -- also when the grid was not fully resident (the host then reports the error).
#pragma once

namespace ct {

// Returns true when the barrier completed, false when the error flag is (or became) raised.
template <typename Ops>
__host__ __device__ inline bool grid_barrier(Ops &ops, int *state, int nblocks, unsigned spin_limit)
{
    ops.block_sync();
    if (ops.leader()) {
        int err = ops.load(&state[3]);
        if (!err) {
            const int gen = ops.load(&state[2]);
            ops.release();
            const int arrived = ops.fetch_add(&state[1], 1) + 1;
            if (arrived == nblocks) {
                ops.store(&state[1], 0);
                ops.store_release(&state[2], gen + 1);
            } else {
                unsigned spins = 0;
                while (ops.load_acquire(&state[2]) == gen) {
                    ops.pause();
                    if (++spins > spin_limit) {
                        ops.store(&state[3], 1);
                        break;
                    }
                }
            }
            ops.acquire();
            err = ops.load(&state[3]);
        }
        ops.set_block_flag(err);
    }
    ops.block_sync();
    return ops.block_flag() == 0;
}

}  // namespace ct
