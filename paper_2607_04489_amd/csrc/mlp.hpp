// mlp.hpp -- shape and parameter layout of the selector MLP (shared by the
// device kernels and the host forward pass).
#pragma once

#include <cstdint>

#include "eiger.h"

namespace eiger {

constexpr int kIn = EIGER_SEL_FEATURES;
constexpr int kHid = EIGER_MLP_HIDDEN;
constexpr int kOut = EIGER_SEL_CLASSES;

// Offsets (in floats) of the parameter blocks in the flat array.
struct MlpOffsets {
  static constexpr int W1 = 0;
  static constexpr int b1 = W1 + kIn * kHid;
  static constexpr int W2 = b1 + kHid;
  static constexpr int b2 = W2 + kHid * kHid;
  static constexpr int W3 = b2 + kHid;
  static constexpr int b3 = W3 + kHid * kOut;
  static constexpr int end = b3 + kOut;
};
constexpr int64_t kParams = MlpOffsets::end;
static_assert(kParams == 6288, "parameter count");

}  // namespace eiger
