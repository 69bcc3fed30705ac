// Part 0 of rda_kernels.inl: table generators, corner turn, unfused comparator kernels, dispatch.
#define SAR_PART 0
#include "rda_kernels.inl"
