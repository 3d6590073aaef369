// Node kernels instantiated for BF16 storage, FP32 arithmetic.
#include "lbm_device.hpp"
#define STGV_T stgv::bf16_t
#define STGV_C float
#define STGV_LAYOUT_KERNELS
#include "lbm_instances.hpp"
