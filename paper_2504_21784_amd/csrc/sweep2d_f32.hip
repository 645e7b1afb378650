// 2D sweep kernels, FP32 instances (the kernel is in sweep2d.inc).
#include "sweep2d.inc"

namespace smrt {
template void launch_sweep2d<float>(const SweepLaunch &, hipStream_t);
}
