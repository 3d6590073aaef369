// Node kernels instantiated for FP16 storage, FP32 arithmetic.
#include "lbm_device.hpp"
#define STGV_T _Float16
#define STGV_C float
#define STGV_LAYOUT_KERNELS
#include "lbm_instances.hpp"
