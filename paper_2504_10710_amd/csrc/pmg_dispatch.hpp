// pmg_dispatch.hpp -- compile-time dispatch of (dimension, degree, type)
// to kernel template instances.
#pragma once

#include "pmg_internal.hpp"


#define PMG_DISPATCH_P(dim, p, ...)                                   \
    do {                                                               \
        if (dim == 2) {                                                \
            switch (p) {                                               \
            case 2: { constexpr int P_ = 2, D_ = 2; __VA_ARGS__; } break;     \
            case 4: { constexpr int P_ = 4, D_ = 2; __VA_ARGS__; } break;     \
            case 8: { constexpr int P_ = 8, D_ = 2; __VA_ARGS__; } break;     \
            case 16: { constexpr int P_ = 16, D_ = 2; __VA_ARGS__; } break;   \
            case 32: { constexpr int P_ = 32, D_ = 2; __VA_ARGS__; } break;   \
            case 64: { constexpr int P_ = 64, D_ = 2; __VA_ARGS__; } break;   \
            case 128: { constexpr int P_ = 128, D_ = 2; __VA_ARGS__; } break; \
            case 256: { constexpr int P_ = 256, D_ = 2; __VA_ARGS__; } break; \
            default: return hipErrorInvalidValue;                      \
            }                                                          \
        } else if (dim == 3) {                                         \
            switch (p) {                                               \
            case 2: { constexpr int P_ = 2, D_ = 3; __VA_ARGS__; } break;     \
            case 4: { constexpr int P_ = 4, D_ = 3; __VA_ARGS__; } break;     \
            case 8: { constexpr int P_ = 8, D_ = 3; __VA_ARGS__; } break;     \
            case 16: { constexpr int P_ = 16, D_ = 3; __VA_ARGS__; } break;   \
            case 32: { constexpr int P_ = 32, D_ = 3; __VA_ARGS__; } break;   \
            case 64: { constexpr int P_ = 64, D_ = 3; __VA_ARGS__; } break;   \
            default: return hipErrorInvalidValue;                      \
            }                                                          \
        } else {                                                       \
            return hipErrorInvalidValue;                               \
        }                                                              \
    } while (0)

// 2-D degrees 4..256 only (levels of several elements per axis)
#define PMG_DISPATCH_P2D(p, ...)                                      \
    do {                                                               \
        switch (p) {                                                   \
        case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;          \
        case 8: { constexpr int P_ = 8; __VA_ARGS__; } break;          \
        case 16: { constexpr int P_ = 16; __VA_ARGS__; } break;        \
        case 32: { constexpr int P_ = 32; __VA_ARGS__; } break;        \
        case 64: { constexpr int P_ = 64; __VA_ARGS__; } break;        \
        case 128: { constexpr int P_ = 128; __VA_ARGS__; } break;      \
        case 256: { constexpr int P_ = 256; __VA_ARGS__; } break;      \
        default: return hipErrorInvalidValue;                          \
        }                                                              \
    } while (0)

// 3-D degrees 4..64 only (levels of several elements per axis)
#define PMG_DISPATCH_P3D(p, ...)                                      \
    do {                                                               \
        switch (p) {                                                   \
        case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;          \
        case 8: { constexpr int P_ = 8; __VA_ARGS__; } break;          \
        case 16: { constexpr int P_ = 16; __VA_ARGS__; } break;        \
        case 32: { constexpr int P_ = 32; __VA_ARGS__; } break;        \
        case 64: { constexpr int P_ = 64; __VA_ARGS__; } break;        \
        default: return hipErrorInvalidValue;                          \
        }                                                              \
    } while (0)

// same, p >= 4 only (operations that need a coarser level)
#define PMG_DISPATCH_P4(dim, p, ...)                                  \
    do {                                                               \
        if (p < 4) return hipErrorInvalidValue;                        \
        if (dim == 2) {                                                \
            switch (p) {                                               \
            case 4: { constexpr int P_ = 4, D_ = 2; __VA_ARGS__; } break;     \
            case 8: { constexpr int P_ = 8, D_ = 2; __VA_ARGS__; } break;     \
            case 16: { constexpr int P_ = 16, D_ = 2; __VA_ARGS__; } break;   \
            case 32: { constexpr int P_ = 32, D_ = 2; __VA_ARGS__; } break;   \
            case 64: { constexpr int P_ = 64, D_ = 2; __VA_ARGS__; } break;   \
            case 128: { constexpr int P_ = 128, D_ = 2; __VA_ARGS__; } break; \
            case 256: { constexpr int P_ = 256, D_ = 2; __VA_ARGS__; } break; \
            default: return hipErrorInvalidValue;                      \
            }                                                          \
        } else if (dim == 3) {                                         \
            switch (p) {                                               \
            case 4: { constexpr int P_ = 4, D_ = 3; __VA_ARGS__; } break;     \
            case 8: { constexpr int P_ = 8, D_ = 3; __VA_ARGS__; } break;     \
            case 16: { constexpr int P_ = 16, D_ = 3; __VA_ARGS__; } break;   \
            case 32: { constexpr int P_ = 32, D_ = 3; __VA_ARGS__; } break;   \
            case 64: { constexpr int P_ = 64, D_ = 3; __VA_ARGS__; } break;   \
            default: return hipErrorInvalidValue;                      \
            }                                                          \
        } else {                                                       \
            return hipErrorInvalidValue;                               \
        }                                                              \
    } while (0)

#define PMG_TYPED(f32, ...)                              \
    do {                                                 \
        if (f32) { using T_ = float; __VA_ARGS__; }      \
        else { using T_ = double; __VA_ARGS__; }         \
    } while (0)

namespace pmg {
static inline hipError_t last() { return hipGetLastError(); }
}  // namespace pmg
