// Internal interface between the operator library and the learned
// preconditioner (a per-patch convolutional network on the spline
// coefficient grid).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

struct igb_cnn;

// Sets the thread-local message returned by igb_last_error().
void igb_set_error(const std::string &msg);

// z = y + f(y) with y = v / D elementwise, for n_img patch grids of h x w
// coefficients each (n = n_img * h * w, image-major, rows of w); f is the
// network in FP32 with BF16 weights.  v, D, z are FP64 device vectors; the
// work is ordered on `st`.  Returns an igb_status.
int32_t cnn_precondition(const igb_cnn *net, int32_t n_img, int32_t h, int32_t w, const double *v, const double *D,
                         double *z, hipStream_t st);

// Training with a loss computed outside the network: a forward pass over a
// batch keeping the activations (*f_out = the correction f, n_img*h*w floats;
// *dout = the buffer of the same size the caller fills with dL/df), then the
// backward pass from *dout and one Adam step.  Both ordered on `st`.
int32_t cnn_batch_forward(igb_cnn *net, const float *in, int32_t n_img, int32_t h, int32_t w, hipStream_t st,
                          float **f_out, float **dout);
int32_t cnn_batch_backward_adam(igb_cnn *net, const float *in, int32_t n_img, int32_t h, int32_t w, float lr,
                                hipStream_t st);
