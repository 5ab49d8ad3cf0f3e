// Host-side helpers of the C-ABI implementation: HIP error propagation,
// device allocation, and the guard that turns exceptions into status codes.
#pragma once

#include <hip/hip_runtime.h>

#include <new>
#include <string>

#include "context.hpp"

namespace fmmkmc {

struct HipError {
    std::string what;
};

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) throw HipError{std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// message of the last failed create call (context or batch) on this thread
inline std::string &create_error()
{
    static thread_local std::string msg;
    return msg;
}

inline int fail(fmmkmc_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

template <typename T>
T *dalloc(size_t count)
{
    if (count == 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(T) * count);
    if (e != hipSuccess) throw std::bad_alloc();
    return (T *)p;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

template <typename T>
void upload(T *dst, const T *src, size_t count, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s));
}

}  // namespace fmmkmc

#define API_GUARD(c, ...)                                            \
    try {                                                            \
        __VA_ARGS__                                                  \
    } catch (const HipError &e) {                                    \
        return fail(c, FMMKMC_EHIP, e.what);                         \
    } catch (const std::bad_alloc &) {                               \
        return fail(c, FMMKMC_ENOMEM, "device or host allocation failed"); \
    }

