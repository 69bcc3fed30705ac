// Part 2 of rda_kernels.inl: line and RCMC kernels with split-FP16 MFMA butterflies.
#define SAR_PART 2
#define SAR_LINE_BATCH_FN launch_line_batch_p2
#include "rda_kernels.inl"
