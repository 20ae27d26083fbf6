// Convolutional surrogate internals shared by conv.hip and the C ABI.
#pragma once

#include "tbh_internal.h"

namespace tbh {

struct Net {
    static constexpr int MAX_LAYERS = 8;
    Ctx* ctx;
    int C;                    // hidden channels
    int CI;                   // input channels
    int L;                    // convolution layers
    int dil[MAX_LAYERS];      // dilation of each layer
    int g[3];                 // nx, ny, nz
    int64_t nvox = 0;
    int64_t n_params = 0;
    int64_t off_w[MAX_LAYERS], off_b[MAX_LAYERS];
    int lin[MAX_LAYERS], lout[MAX_LAYERS];
    DevBuf w32, m32, v32, grad, w16, wt16, xin, pred, part, dpart, scalar, lw, counts;
    DevBuf act[MAX_LAYERS], dact[2];   // act[l]: output of layer l < L-1 (FP16)
    bool weighted = false;             // lw holds per-voxel loss weights
    int nchunk = 1;
    int step_t = 0;
    Net(Ctx* c, int channels, int in_channels, int n_layers, const int* dilations, const int grid[3]);
    void set_loss_weights(const float* w_dev);           // [nvox] FP32 copied, or null = uniform
    void zero_moments();
    void sync_half();                                    // FP16 copies of the FP32 masters
    void forward(const float* x_dev, float* y_dev);      // x: [CI][nvox]; y_dev null: into pred
    double accumulate_gradients(const float* x_dev, const float* t_dev);  // returns the sample's MSE
    void zero_grad();
    bool adam(double lr, int batch);   // false: skipped (non-finite gradient)
};

}  // namespace tbh
