// Node kernels instantiated for FP32 storage, FP64 arithmetic.
#include "lbm_device.hpp"
#define STGV_T float
#define STGV_C double
#include "lbm_instances.hpp"
