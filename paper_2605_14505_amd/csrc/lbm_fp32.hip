// Node kernels instantiated for FP32 storage, FP32 arithmetic.
#include "lbm_device.hpp"
#define STGV_T float
#define STGV_C float
#define STGV_LAYOUT_KERNELS
#include "lbm_instances.hpp"
