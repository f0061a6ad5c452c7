// launch_rules.hpp -- host-side launch-size rules of libsbr kernels.
// Plain C++ with no HIP dependency, so that the rules can be checked on a
// machine without a GPU.
#pragma once
#include <cstddef>

namespace sbr {

constexpr int kWaveLanes = 64;
// LDS a workgroup may allocate (bytes)
constexpr std::size_t kReplayLdsMax = 65536;

// Threads per block of the capture replay: the tuned size, lowered in whole
// waves until the block's traversal stacks (stack_bytes per thread, in LDS)
// fit kReplayLdsMax.  A single wave is the floor.
inline int replay_block_for(int tuned, std::size_t stack_bytes) {
  int rb = tuned;
  while (rb > kWaveLanes && (std::size_t)rb * stack_bytes > kReplayLdsMax) rb -= kWaveLanes;
  return rb;
}

}  // namespace sbr
