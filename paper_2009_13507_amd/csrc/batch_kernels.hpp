// batch_kernels.hpp -- persistent batched imaginary-time stepping.
#pragma once
#include "step_kernels.hpp"
