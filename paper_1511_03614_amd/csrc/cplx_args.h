// Kernel argument of the complex-mode evaluators, shared by the host launchers
// and the HIP kernels (plain C++).
#pragma once
#include <stdint.h>

#include "sdint_internal.h"

namespace sdi {

struct CplxArgs {
  const CplxDev* cx;        // [nsec] (tile kernel) or the evaluated sector's record
  const uint32_t* dir;      // derivative-list directory
};

}  // namespace sdi
