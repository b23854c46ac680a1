// rst_cnn_api.hpp -- host interface of the learned correction network (the
// kernels are in rst_cnn.hpp, the driver in rst_cnn.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rst {
namespace cnn {

// Natural weight layout: layers W0..W8 one after another, each (cout, cin, 3, 3, 3)
// row-major with the taps ordered (dz, db, da), each offset -1..1, dz slowest.
// (cout, cin): W0 (16, 4), W1..W7 (16, 16), W8 (2, 16).
constexpr int kLayerCin[9] = {4, 16, 16, 16, 16, 16, 16, 16, 16};
constexpr int kLayerCout[9] = {16, 16, 16, 16, 16, 16, 16, 16, 2};
size_t natural_count();  // 50976

class Engine;
Engine* engine_create(hipStream_t s);
void engine_destroy(Engine* e);
hipError_t engine_seed(Engine* e, uint64_t seed);  // He-normal weights, last layer x0.1
hipError_t engine_set_weights(Engine* e, const float* natural_host);
hipError_t engine_get_weights(Engine* e, float* natural_host);
// f(x) for ncol columns on an (nz, nb, na) grid: x [ncol][n][4], out [ncol][n][2]
// (device).  keep = true keeps the activations for engine_backward.
hipError_t engine_forward(Engine* e, const float* x, float* out, int ncol, int nz, int nb, int na, bool keep);
// weight gradient of <gout, f(x)> for the x of the last kept forward; gout
// [ncol][n][4] with channels 2, 3 zero.  Result kept on the device.
hipError_t engine_backward(Engine* e, const float* gout4);
hipError_t engine_get_grad(Engine* e, float* natural_host);
// loss = mean over columns of ||out - tgt||^2 and gout4 = 2 (out - tgt) / ncol
hipError_t engine_loss(Engine* e, const float* out, const float* tgt, float* gout4, int ncol, long long n,
                       double* loss);
hipError_t engine_adam(Engine* e, float lr);
// weight gradient of <g, f(x)> with a two-channel g [ncol][n][2] (device)
hipError_t engine_gradient(Engine* e, const float* x, const float* g2, int ncol, int nz, int nb, int na);
// one Adam step on the loss of (x, tgt); loss before the step into *loss
hipError_t engine_train_step(Engine* e, const float* x, const float* tgt, int ncol, int nz, int nb, int na,
                             float lr, double* loss);
void engine_reset_adam(Engine* e);
bool engine_has_weights(const Engine* e);

}  // namespace cnn
}  // namespace rst
