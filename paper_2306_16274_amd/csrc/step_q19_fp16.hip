// Step kernels of D3Q19 with fp16 storage (one translation unit per pair, compiled in parallel).
#include "step_ops.h"

template struct StepOps<19, _Float16>;
