// FP32 instantiation of the generic kernels (FP64 geometry, FP32 contraction).
#define GEN_T float
#define GEN_SUFFIX select_generic_f32
#include "k_generic.inl"
