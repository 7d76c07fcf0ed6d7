// fj_guard.hpp -- how the C ABI keeps C++ exceptions inside the library.
//
// Host-only C++ (no HIP): every int-returning entry point of fj_api.hip runs
// its body through guarded(), so that a C++ exception -- a failed host
// allocation in a std container or operator new, or anything else -- becomes
// a status code and a message in the calling thread's error buffer instead of
// unwinding through the C ABI (which would terminate a C or ctypes caller).
#pragma once

#include <cstdio>
#include <exception>
#include <new>

#include "../../include/fj.h"

namespace fj {

// Detail of the last error on this thread (fj_last_error).
inline thread_local char g_last_error[256] = "";

template <typename F>
int guarded(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        std::snprintf(g_last_error, sizeof g_last_error, "host memory allocation failed");
        return FJ_ERR_HOST_MEMORY;
    } catch (const std::exception& e) {
        std::snprintf(g_last_error, sizeof g_last_error, "C++ exception: %s", e.what());
        return FJ_ERR_INTERNAL;
    } catch (...) {
        std::snprintf(g_last_error, sizeof g_last_error, "unknown C++ exception");
        return FJ_ERR_INTERNAL;
    }
}

}  // namespace fj
