// Convolutional surrogate internals shared by conv.hip and the C ABI.
#pragma once

#include "tbh_internal.h"

namespace tbh {

struct Net {
    Ctx* ctx;
    int C;                    // hidden channels
    int CI;                   // input channels
    int g[3];                 // nx, ny, nz
    int64_t nvox = 0;
    int64_t n_params = 0;
    int64_t off_w[4], off_b[4];
    int lin[4], lout[4];
    DevBuf w32, m32, v32, grad, w16, wt16, xin, pred, part, dpart, scalar;
    DevBuf act[4], dact[2];
    int nchunk = 1;
    int step_t = 0;
    Net(Ctx* c, int channels, int in_channels, const int grid[3]);
    void zero_moments();
    void sync_half();                                    // FP16 copies of the FP32 masters
    void forward(const float* x_dev, float* y_dev);      // x: [CI][nvox]; y_dev null: into pred
    double accumulate_gradients(const float* x_dev, const float* t_dev);  // returns the sample's MSE
    void zero_grad();
    void adam(double lr, int batch);
};

}  // namespace tbh
