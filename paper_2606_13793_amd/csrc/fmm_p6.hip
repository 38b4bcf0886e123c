// Kernels and launch code of the FMM solve for expansion order p = 6.
#include "fmm_impl.h"

template struct fmm::Impl<6>;
