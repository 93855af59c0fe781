// FP64 instantiation of the generic kernels.
#define GEN_T double
#define GEN_SUFFIX select_generic_f64
#include "k_generic.inl"
