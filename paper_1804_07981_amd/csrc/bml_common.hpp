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

// Helper launches shared by the single-lattice and batch code (defined in
// bml_lattice.hip).  All are asynchronous on `stream`.  A lattice has `rows`
// rows of `cols` cells (cols a multiple of 32).
// Random initial state (layout 0 = bytes, 1 = planes): cell k is LR w.p.
// rho_lr and TB w.p. rho_tb (rho/2 each for the symmetric draw).
int launch_init(void *state, int32_t rows, int32_t cols, int32_t layout, uint64_t seed,
                double rho_lr, double rho_tb, hipStream_t stream);
// counts[0] = LR cars, counts[1] = TB cars of the state (clears them first).
int launch_count(const void *state, int32_t rows, int32_t cols, int32_t layout,
                 unsigned long long *counts, hipStream_t stream);
int launch_pack(const uint8_t *cells, uint32_t *planes, int32_t rows, int32_t cols,
                hipStream_t stream);
int launch_unpack(const uint32_t *planes, uint8_t *cells, int32_t rows, int32_t cols,
                  hipStream_t stream);
// n_words words of the LR plane `lr` and the TB plane `tb` -> 32 n_words
// byte cells.
int launch_unpack_rows(const uint32_t *lr, const uint32_t *tb, uint8_t *cells, int64_t n_words,
                       hipStream_t stream);
int launch_zero(uint32_t *p, int64_t words, hipStream_t stream);

inline bool valid_n(int32_t n) { return n >= 32 && n <= 65504 && n % 32 == 0; }
// Rectangular lattices: 32..65504 rows (any count) of 32..65504 cells (a
// multiple of 32), so every byte offset stays below 2^32.
inline bool valid_shape(int32_t rows, int32_t cols)
{
    return rows >= 32 && rows <= 65504 && valid_n(cols);
}

} // namespace bml
