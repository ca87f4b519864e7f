// Stand-in of <hip/hip_ext.h> for the host-only build (see hip_runtime.h).
#pragma once
#include "hip_runtime.h"
