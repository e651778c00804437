// bml_common.hpp -- host-side helpers shared by the libbml translation units:
// error reporting, HIP call checking and device properties.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include "bml.h"

namespace bml {

// Records a printf-style message as the calling thread's last error and
// returns `code`.
int fail(int code, const char *fmt, ...);
void clear_error();

#define BML_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::bml::fail(BML_EDEVICE, "%s failed: %s", #call,                \
                               hipGetErrorString(e_));                             \
    } while (0)

struct DeviceInfo {
    int device = -1;
    int cu_count = 0;
};

// Properties of the current device (cached per device).
int device_info(DeviceInfo *out);

inline bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

inline bool valid_n(int32_t n) { return n >= 32 && n <= 65504 && n % 32 == 0; }

} // namespace bml
