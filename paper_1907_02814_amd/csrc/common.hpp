// common.hpp -- error reporting and the table handle shared by the
// translation units of libcmc.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "../../include/cmc.h"
#include "tabview.hpp"

struct cmc_tables_s {
    int Z;
    int device;
    double Ltf, fc;
    cmc::Axes ax;
    double* d64;                              // all arrays, FP64
    float* d32;                               // all arrays, FP32
    long long off[cmc::grid::kNumArrays];     // element offsets of each array
    long long total;
};

namespace cmc {

void set_error(const char* fmt, ...);

// FP64 / FP32 views of a table handle
TabView<double> view64(const cmc_tables_s* t);
TabView<float> view32(const cmc_tables_s* t);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace cmc

#define CMC_CHECK_LAUNCH(what)                                                   \
    do {                                                                         \
        hipError_t e_ = hipGetLastError();                                       \
        if (e_ != hipSuccess) {                                                  \
            cmc::set_error("%s: %s", what, hipGetErrorString(e_));               \
            return CMC_EDEVICE;                                                  \
        }                                                                        \
    } while (0)

#define CMC_CHECK_LAUNCH2(who, what)                                             \
    do {                                                                         \
        hipError_t e_ = hipGetLastError();                                       \
        if (e_ != hipSuccess) {                                                  \
            cmc::set_error("%s: %s: %s", who, what, hipGetErrorString(e_));      \
            return CMC_EDEVICE;                                                  \
        }                                                                        \
    } while (0)

#define CMC_REQUIRE(cond, code, ...)                                             \
    do {                                                                         \
        if (!(cond)) { cmc::set_error(__VA_ARGS__); return code; }               \
    } while (0)

namespace cmc {
// NULL, or aligned to the element type the library reads there (the host
// check of a device array pointer; nothing is dereferenced)
template <typename T>
inline bool aligned_to(const void* p) {
    return (reinterpret_cast<uintptr_t>(p) % alignof(T)) == 0;
}
}  // namespace cmc
