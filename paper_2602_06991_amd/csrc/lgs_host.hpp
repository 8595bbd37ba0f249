// Host-side plumbing shared by the C-ABI entry points: the per-thread error
// message, argument checks and launch checks.  No exception leaves an entry point.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "lgs.h"

namespace lgs {

void set_error(const char *fmt, ...);
void clear_error();

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline bool k_supported(int k) {
    switch (k) {
    case 1: case 2: case 3: case 4: case 5: case 8: case 10: case 16: return true;
    default: return false;
    }
}

inline lgs_status check_camera(const lgs_camera *cam) {
    if (!cam) { set_error("camera is NULL"); return LGS_ERR_INVALID_ARG; }
    if (cam->width <= 0 || cam->height <= 0 || cam->width > 32768 || cam->height > 32768) {
        set_error("camera size %dx%d out of range", cam->width, cam->height);
        return LGS_ERR_INVALID_ARG;
    }
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) {
        set_error("camera focal lengths must be positive");
        return LGS_ERR_INVALID_ARG;
    }
    return LGS_OK;
}

inline lgs_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return LGS_ERR_HIP;
    }
    return LGS_OK;
}

inline lgs_status check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return LGS_ERR_HIP;
    }
    return LGS_OK;
}

#define LGS_REQUIRE(cond, code, ...)          \
    do {                                      \
        if (!(cond)) {                        \
            ::lgs::set_error(__VA_ARGS__);    \
            return code;                      \
        }                                     \
    } while (0)

inline int tiles_x(int w) { return (w + LGS_TILE - 1) / LGS_TILE; }
inline int tiles_y(int h) { return (h + LGS_TILE - 1) / LGS_TILE; }

// Grid padded to a multiple of 8 blocks for the XCD remap.
inline unsigned padded_grid(long long blocks) { return (unsigned)(((blocks + 7) / 8) * 8); }

}  // namespace lgs
