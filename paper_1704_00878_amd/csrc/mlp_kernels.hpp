// Learned center proposer kernels (filled in below).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
