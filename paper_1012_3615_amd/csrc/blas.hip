// BLAS-1 kernels (placeholder).
#include "kernels.h"
