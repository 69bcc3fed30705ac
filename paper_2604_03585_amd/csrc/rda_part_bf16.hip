// Part 3 of rda_kernels.inl: line and RCMC kernels with split-BF16 MFMA butterflies.
#define SAR_PART 3
#define SAR_LINE_BATCH_FN launch_line_batch_p3
#include "rda_kernels.inl"
