// Step kernels of D3Q27 with fp32 storage (one translation unit per pair, compiled in parallel).
#include "step_ops.h"

template struct StepOps<27, float>;
