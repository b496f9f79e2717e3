// Bounded host-side waits for device work.
//
// A host thread that waits for the GPU (the plan's readback, a server
// worker's batch, a tuner's timing run) polls a completion query instead of
// sleeping in a runtime synchronisation, so it returns as soon as the work is
// done.  The poll is bounded and polite:
//   - it gives up after a wall-clock limit, so a device that stalls becomes
//     an HP_ERR_TIMEOUT status instead of a host thread that never returns;
//   - after a short burst of back-to-back polls it yields the core between
//     polls, and after a longer burst it sleeps between polls, so waiting
//     threads do not pin host cores.
// Header-only and free of HIP types: the host test-suite drives it with a
// fake query and a fake clock.
#pragma once

#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <thread>

namespace hp {

enum class Poll : int { READY = 0, PENDING = 1, FAILED = 2 };
enum class WaitResult : int { DONE = 0, FAILED = 1, TIMED_OUT = 2 };

struct WaitPolicy {
    int64_t limit_ns;   // give up once this much time has passed (<= 0: never)
    int spin_polls;     // polls back to back before the first pause
    int yield_polls;    // then polls separated by a yield of the core
    int64_t sleep_ns;   // then polls separated by a sleep of this length
};

// Limit of every host wait: the environment variable HP_HOST_WAIT_MS when
// it holds a positive number, else ten minutes.
inline int64_t host_wait_limit_ns() {
    const char *s = std::getenv("HP_HOST_WAIT_MS");
    if (s) {
        char *end = nullptr;
        const long long ms = std::strtoll(s, &end, 10);
        if (end != s && ms > 0) return (int64_t)ms * 1000000;
    }
    return int64_t(600) * 1000000000;
}

inline WaitPolicy default_wait_policy() { return WaitPolicy{host_wait_limit_ns(), 256, 2048, 20000}; }

// Polls query() (returning Poll) until READY or FAILED, or until now() has
// advanced limit_ns past its first reading.  pause(ns) is called between
// polls once the spin burst is over: ns == 0 asks for a yield, ns > 0 for a
// sleep.  *polls (optional) receives the number of queries made.
template <class Query, class Now, class Pause>
WaitResult wait_until(Query query, const WaitPolicy &pol, Now now, Pause pause, int64_t *polls = nullptr) {
    const int64_t t0 = now();
    for (int64_t k = 0;; k++) {
        const Poll s = query();
        if (polls) *polls = k + 1;
        if (s == Poll::READY) return WaitResult::DONE;
        if (s == Poll::FAILED) return WaitResult::FAILED;
        if (pol.limit_ns > 0 && now() - t0 >= pol.limit_ns) return WaitResult::TIMED_OUT;
        if (k + 1 < pol.spin_polls) continue;
        pause(k + 1 < (int64_t)pol.spin_polls + pol.yield_polls ? 0 : pol.sleep_ns);
    }
}

inline int64_t steady_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

inline void pause_ns(int64_t ns) {
    if (ns <= 0) std::this_thread::yield();
    else std::this_thread::sleep_for(std::chrono::nanoseconds(ns));
}

// The same with the steady clock and real yields and sleeps.
template <class Query>
WaitResult wait_until(Query query, const WaitPolicy &pol) {
    return wait_until(query, pol, steady_ns, pause_ns);
}

}  // namespace hp
