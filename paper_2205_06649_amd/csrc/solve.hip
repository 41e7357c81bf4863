// Placeholder translation unit for the batched L-BFGS kernels.
#include <hip/hip_runtime.h>
