// Step kernels of D3Q27 with fp16 storage (one translation unit per pair, compiled in parallel).
#include "step_ops.h"

template struct StepOps<27, _Float16>;
