// Part 1 of rda_kernels.inl: line and RCMC kernels with FP32 butterflies.
#define SAR_PART 1
#define SAR_LINE_BATCH_FN launch_line_batch_p1
#include "rda_kernels.inl"
