// Host stand-ins for the device launchers of build.hip, step.hip and read.hip,
// for the ThreadSanitizer build of the library's host files: no kernel runs;
// the build publishes consistent reverse-row column starts and each step
// advances the host clock and consolidation count exactly as the real
// launchers do, after a short sleep that lets the server's threads
// interleave.
#include <hip/hip_runtime.h>

#include <chrono>
#include <thread>

#include "net.h"

namespace dpsnn {

void Timers::collect() { pending.clear(); }
void Timers::release() { pool.clear(); pending.clear(); }

hipError_t launch_build(Net& n) {
    for (uint32_t c = 0; c <= n.d.C; ++c) n.col_rev_dev[c] = n.S_exc * c / n.d.C;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
    return hipSuccess;
}

hipError_t launch_step_set(LaunchSet& L, const Tuning&, Timers&, hipStream_t, Net* const* members) {
    for (uint32_t k = 0; k < L.K; ++k) {
        Net& n = *members[k];
        const uint32_t T = n.cfg.weight_update_period;
        if (T && (n.t + 1) % T == 0) n.consolidations++;
        n.t += 1;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100));
    return hipSuccess;
}

hipError_t launch_steps(LaunchSet& L, const Tuning& tune, Timers& tm, hipStream_t s, Net* const* members,
                        uint32_t n_steps) {
    for (uint32_t i = 0; i < n_steps; ++i) {
        const hipError_t e = launch_step_set(L, tune, tm, s, members);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_read_rows(Net&, uint32_t, uint32_t, uint64_t, uint64_t, const float*, uint64_t,
                            uint32_t*, uint8_t*, float*, float*, float*) {
    return hipSuccess;
}
hipError_t launch_P_to_forward(Net&, float*, uint32_t, uint32_t, bool) { return hipSuccess; }
hipError_t launch_P_from_forward(Net&, float*, uint32_t, uint32_t) { return hipSuccess; }

}  // namespace dpsnn
