// Single translation unit of the HIP library (gfx950): every kernel and the
// C ABI are compiled together so kernels and their launch sites share one
// code object.
#include "internal.hpp"
#include "build.hip"
#include "factor.hip"
#include "factor_mwg.hip"
#include "solve.hip"
#include "gmres.hip"
#include "fft.hip"
#include "adi.hip"
#include "ek.hip"
#include "convnet.hip"
#include "api.hip"
#include "api2d.hip"
#include "apinet.hip"
