// Threads for the host-side builders (C++17, no HIP).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdlib>
#include <exception>
#include <thread>
#include <vector>

namespace sem {

// Worker threads for the host build: SEM_HOST_THREADS when set (for any
// mesh size); else the process's CPU share as the OpenMP convention states
// it (OMP_NUM_THREADS) when set, else the hardware count, at most 32, and
// one thread for small meshes.  The tables do not depend on the count.
inline int host_threads(size_t work) {
    if (const char* e = std::getenv("SEM_HOST_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0) return std::min(v, 32);
    }
    if (work < (size_t(1) << 16)) return 1;
    int n = int(std::thread::hardware_concurrency());
    if (const char* e = std::getenv("OMP_NUM_THREADS")) {
        const int v = std::atoi(e);
        if (v > 0) n = v;
    }
    return std::max(1, std::min(n, 32));
}

// f(begin, end, t) over T contiguous ranges of [0, n), one thread each.  A
// range whose thread cannot be started runs on the calling thread; the first
// exception of any range is rethrown once every thread has joined.
template <typename F>
inline void parallel_ranges(size_t n, int T, F f) {
    if (T <= 1) {
        f(size_t(0), n, 0);
        return;
    }
    std::vector<std::exception_ptr> err(static_cast<size_t>(T));
    auto run = [&f, &err](size_t b, size_t e, int t) {
        try {
            f(b, e, t);
        } catch (...) {
            err[size_t(t)] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve(size_t(T));
    for (int t = 0; t < T; ++t) {
        const size_t b = n * size_t(t) / size_t(T), e = n * size_t(t + 1) / size_t(T);
        try {
            th.emplace_back(run, b, e, t);
        } catch (...) {
            run(b, e, t);
        }
    }
    for (auto& x : th) x.join();
    for (auto& x : err)
        if (x) std::rethrow_exception(x);
}

}  // namespace sem
