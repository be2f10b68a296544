// Transform lengths served by the library: powers of two from 16 to 2048
// and 3 * 2^k for 384, 768, 1536. Every length-templated kernel is
// instantiated once per length; the build compiles one column-pass
// translation unit per length (the list there must match).
#pragma once

namespace cip {

constexpr int kSizes[] = {16, 32, 64, 128, 256, 384, 512, 768, 1024, 1536, 2048};

constexpr bool size_supported(int n) {
  for (int s : kSizes)
    if (s == n) return true;
  return false;
}

}  // namespace cip

// X-macro over the lengths (column-pass launcher declarations and cases).
#define CIP_FOR_EACH_SIZE(X) \
  X(16) X(32) X(64) X(128) X(256) X(384) X(512) X(768) X(1024) X(1536) X(2048)

// switch over the runtime length N binding the compile-time constant NN.
#define CIP_DISPATCH_N(N, ...)                                     \
  switch (N) {                                                     \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;        \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;        \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;        \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;      \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;      \
    case 384: { constexpr int NN = 384; __VA_ARGS__; } break;      \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;      \
    case 768: { constexpr int NN = 768; __VA_ARGS__; } break;      \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break;    \
    case 1536: { constexpr int NN = 1536; __VA_ARGS__; } break;    \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; } break;    \
    default: return hipErrorInvalidValue;                          \
  }
