// Host emulation of HIP: the runtime API part (see hip_runtime.h).
// TEST INFRASTRUCTURE ONLY.
#pragma once
#include "hip_runtime.h"
