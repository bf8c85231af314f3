// Learned pointwise preconditioner kernels (filled in below).
#include "common.hpp"
namespace ofks {}
