// Library-owned grid U-Net of the surrogate control step (internal, host side).
//
// The network stands in for one control step of 25 substeps (25 physics
// steps per control step, App. E.3); the library runs its forward pass on the
// per-scene boxes the surrogate works on, with the BF16-MFMA convolution
// kernels of mpm_nn.h, on the context's stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace mpm {

struct SurNet;

// Parse a weight blob (format in include/mpm.h, mpm_surrogate_load), copy it to
// the current device and pack the BF16 fragments on `st`.  Returns nullptr
// and sets *err on failure (err_code: -1 bad blob, -2 HIP error, -3 out of
// memory).
SurNet *surnet_load(const void *blob, size_t bytes, hipStream_t st, std::string *err, int *err_code);
void surnet_destroy(SurNet *net);

int surnet_cin(const SurNet *net);    // input channels the blob was made for (the features give 8)
int surnet_cout(const SurNet *net);   // output channels (>= 4: velocity change, mass change, ...)

// The network on n boxes of D x H x W nodes (multiples of 4): feat
// [n][D][H][W][cf] FP32 (the first cin channels read) -> pred [n][D][H][W][cout]
// FP32.  Activation buffers are (re)allocated when (n, D, H, W) changes.
// Returns 0, -1 on bad sizes, -2 on a HIP error, -3 out of memory.
int surnet_forward(SurNet *net, const float *feat, int cf, int n, int D, int H, int W, float *pred, hipStream_t st,
                   std::string *err);

}  // namespace mpm
