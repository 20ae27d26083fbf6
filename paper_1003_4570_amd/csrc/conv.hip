// 3-D convolutional surrogate of the self-consistent potential: inference
// and training kernels.
//
// The self-consistent loop of the paper (Sec. III-A) iterates from a start
// potential; this network maps input maps derived from the donor layout to a
// start potential.  L 3x3x3 convolutions c_in -> C -> ... -> C -> 1 with a
// dilation per layer (default four layers, dilations (1, 2, 4, 1)), ReLU
// after all but the last, circular padding along x and y, zero padding
// along z.  Activations are FP16, channels-last [voxel][channel]; weights are
// FP32 masters with FP16 copies, laid out [c_out][tap][c_in] with
// tap = dz*9 + dy*3 + dx (offset (d-1)*dilation).
//
// Forward and backward-data are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x16f16, FP32 accumulation): M = 16 voxels per wavefront,
// N = output channels, K = 27 taps x input channels, the A operand gathered
// straight from the shifted voxels (8-byte loads of 4 channels), the B
// operand from the FP16 weights.  Backward-data is the forward convolution
// of the upstream gradient with tap-reversed, channel-transposed weights,
// with the previous layer's ReLU mask applied in the epilogue.  The weight
// gradient is a third implicit GEMM on the matrix cores (K = voxels, staged
// through LDS), reduced over workgroups in fixed order.  The loss
// gradient is scaled by the voxel count (sum of squares) so FP16 gradients
// stay in range; the optimizer divides it back out.
#include <cmath>
#include <vector>

#include "conv.h"
#include "tbh_internal.h"

namespace tbh {

namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int TPB = 256;

struct Geo {
    int nx, ny, nz;
    int64_t nvox;
};

__device__ __forceinline__ int64_t shifted_voxel(const Geo g, int64_t v, int tap, int dil) {
    const int x = int(v % g.nx);
    const int y = int((v / g.nx) % g.ny);
    const int z = int(v / (int64_t(g.nx) * g.ny));
    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
    const int zz = z + (dz - 1) * dil;
    if (zz < 0 || zz >= g.nz) return -1;
    int yy = (y + (dy - 1) * dil) % g.ny;
    if (yy < 0) yy += g.ny;
    int xx = (x + (dx - 1) * dil) % g.nx;
    if (xx < 0) xx += g.nx;
    return (int64_t(zz) * g.ny + yy) * g.nx + xx;
}

// out[v][co] = act(b[co] + sum_{t, ci} W[co][t][ci] in[shift_t(v)][ci])
// MODE 0: ReLU, FP16 out; 1: identity, FP32 out; 2: identity times the mask
// (mask[v][co] > 0), FP16 out (backward-data).
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(TPB) void k_conv(Geo g, int dil, const _Float16* __restrict__ in,
                                              const _Float16* __restrict__ W, const _Float16* __restrict__ bias,
                                              const _Float16* __restrict__ mask, void* out) {
    constexpr int K = 27 * CIN;
    constexpr int KS = (K + 15) / 16;
    constexpr int NT = (COUT + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t v0 = (int64_t(blockIdx.x) * 4 + wave) * 16;
    if (v0 >= g.nvox) return;
    const int row = lane & 15, kq = lane >> 4;
    const int64_t v = v0 + row;
    const bool vin = v < g.nvox;
    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KS; ++ks) {
        const int k0 = ks * 16 + kq * 4;
        h4 a;
        if constexpr (CIN % 4 == 0) {
            const int tap = k0 / CIN, ci = k0 % CIN;
            const int64_t s = (vin && k0 < K) ? shifted_voxel(g, v, tap, dil) : -1;
            if (s >= 0) a = *reinterpret_cast<const h4*>(in + s * CIN + ci);
            else a = h4{0, 0, 0, 0};
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + e;
                _Float16 val = 0;
                if (k < K && vin) {
                    const int tap = k / CIN, ci = k % CIN;
                    const int64_t s = shifted_voxel(g, v, tap, dil);
                    if (s >= 0) val = in[s * CIN + ci];
                }
                a[e] = val;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + row;
            h4 b;
            if constexpr (K % 4 == 0) {
                if (co < COUT && k0 < K) b = *reinterpret_cast<const h4*>(W + int64_t(co) * K + k0);
                else b = h4{0, 0, 0, 0};
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = (co < COUT && k0 + e < K) ? W[int64_t(co) * K + k0 + e] : _Float16(0);
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc[t], 0, 0, 0);
        }
    }
    // D[i = 4*(lane/16) + r][j = lane%16]: voxel v0 + i, channel t*16 + j
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int co = t * 16 + row;
        if (co >= COUT) continue;
        const float bb = bias ? float(bias[co]) : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t vo = v0 + kq * 4 + r;
            if (vo >= g.nvox) continue;
            float val = acc[t][r] + bb;
            if constexpr (MODE == 0) {
                val = val > 0.f ? val : 0.f;
                static_cast<_Float16*>(out)[vo * COUT + co] = _Float16(val);
            } else if constexpr (MODE == 1) {
                static_cast<float*>(out)[vo * COUT + co] = val;
            } else {
                if (!(float(mask[vo * COUT + co]) > 0.f)) val = 0.f;
                static_cast<_Float16*>(out)[vo * COUT + co] = _Float16(val);
            }
        }
    }
}

// Weight gradient on the matrix cores: dW[co][n] = sum_v dout[v][co] in[shift_tap(v)][ci]
// with n = tap * CIN + ci (the [c_out][tap][c_in] layout), and the bias
// gradient as one more column n = 27 CIN whose input is 1 on every voxel.
// As a GEMM: M = output channels, N = 27 CIN + 1, K = voxels.  Each
// workgroup walks chunks of 64 voxels (grid-stride over blockIdx.x); per
// chunk the upstream gradient is staged once into LDS as [co][64 voxels]
// (the A operand, 4 consecutive voxels per 8-byte read), and each wave
// stages, per column tile of 16, the shifted input values as [16][64 voxels]
// (the B operand).  blockIdx.y selects a group of 4 TPW column tiles (TPW per
// wave).  Partial sums stay in the accumulators over the workgroup's chunks
// and are written to part[blockIdx.x][w] (w = co * 27 CIN + n, then the
// biases), which k_reduce_chunks sums over blockIdx.x in fixed order.
template <int CIN, int COUT, int TPW>
__global__ __launch_bounds__(TPB) void k_conv_wgrad(Geo g, int dil, const _Float16* __restrict__ in,
                                                    const _Float16* __restrict__ dout, float* __restrict__ part) {
    constexpr int N = 27 * CIN;             // weight columns; column N is the bias
    constexpr int NW = COUT * N;
    constexpr int COT = (COUT + 15) / 16;   // row tiles
    constexpr int NTN = (N + 1 + 15) / 16;  // column tiles
    __shared__ _Float16 sD[COT * 16][64];
    __shared__ _Float16 sB[TPB / 64][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, c16 = lane & 15;
    const int tile0 = (blockIdx.y * (TPB / 64) + wave) * TPW;
    f4 acc[TPW][COT];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int c = 0; c < COT; ++c) acc[t][c] = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t nchunks = (g.nvox + 63) / 64;
    for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int64_t v0 = ch * 64;
        __syncthreads();   // the previous chunk's LDS reads are done
        for (int idx = threadIdx.x; idx < COT * 16 * 64; idx += TPB) {
            const int co = idx >> 6, vv = idx & 63;
            const int64_t v = v0 + vv;
            sD[co][vv] = (co < COUT && v < g.nvox) ? dout[v * COUT + co] : _Float16(0);
        }
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int n0 = (tile0 + t) * 16;
            // this lane stages voxel v0 + lane for the tile's 16 columns
            const int64_t v = v0 + lane;
            const bool vin = v < g.nvox;
            if constexpr (CIN % 16 == 0) {
                // the tile's 16 columns are 16 consecutive channels of one tap
                const int tap = n0 / CIN, ci0 = n0 % CIN;
                _Float16 vals[16];
                if (n0 < N) {
                    const int64_t sv = vin ? shifted_voxel(g, v, tap, dil) : -1;
                    if (sv >= 0) {
                        const h4* src = reinterpret_cast<const h4*>(in + sv * CIN + ci0);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const h4 x = src[e];
#pragma unroll
                            for (int u = 0; u < 4; ++u) vals[4 * e + u] = x[u];
                        }
                    } else {
#pragma unroll
                        for (int jj = 0; jj < 16; ++jj) vals[jj] = _Float16(0);
                    }
                } else {
#pragma unroll
                    for (int jj = 0; jj < 16; ++jj) vals[jj] = (n0 + jj == N && vin) ? _Float16(1) : _Float16(0);
                }
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) sB[wave][jj][lane] = vals[jj];
            } else {
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const int n = n0 + jj;
                    _Float16 val = 0;
                    if (vin && n < N) {
                        const int64_t sv = shifted_voxel(g, v, n / CIN, dil);
                        if (sv >= 0) val = in[sv * CIN + n % CIN];
                    } else if (vin && n == N) {
                        val = 1;
                    }
                    sB[wave][jj][lane] = val;
                }
            }
            __syncthreads();   // sD and this tile's sB are staged
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const h4 b = *reinterpret_cast<const h4*>(&sB[wave][c16][ks * 16 + 4 * q]);
#pragma unroll
                for (int c = 0; c < COT; ++c) {
                    const h4 a = *reinterpret_cast<const h4*>(&sD[c * 16 + c16][ks * 16 + 4 * q]);
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc[t][c], 0, 0, 0);
                }
            }
            __syncthreads();   // sB is free for the next tile
        }
    }
    // D[i = 4 q + r][j = c16]: output channel c * 16 + 4 q + r, column tile * 16 + c16
    float* out = part + int64_t(blockIdx.x) * (NW + COUT);
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int n = (tile0 + t) * 16 + c16;
        if (tile0 + t >= NTN || n > N) continue;
#pragma unroll
        for (int c = 0; c < COT; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = c * 16 + 4 * q + r;
                if (co >= COUT) continue;
                out[n < N ? co * N + n : NW + co] = acc[t][c][r];
            }
    }
}

// grad[w] += sum over chunks (fixed order)
__global__ void k_reduce_chunks(const float* part, int nchunk, int nw, float* grad) {
    const int w = blockIdx.x * TPB + threadIdx.x;
    if (w >= nw) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[int64_t(c) * nw + w];
    grad[w] += float(s);
}

// pred FP32, target FP32, optional per-voxel weight w (null = 1): partial sum
// of w (pred - target)^2, dout = 2 w (pred - target) in FP16
__global__ void k_mse(int64_t n, const float* pred, const float* target, const float* w, _Float16* dout,
                      double* part) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        const float d = pred[i] - target[i];
        const float wi = w ? w[i] : 1.f;
        dout[i] = _Float16(2.f * wi * d);
        acc += double(wi) * double(d) * double(d);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_sum_part(const double* part, int n, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s;
    }
}

// [cin][nvox] FP32 -> [nvox][cin] FP16
__global__ void k_pack_input(int64_t nvox, int cin, const float* a, _Float16* b) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < nvox; i += int64_t(gridDim.x) * TPB)
        for (int c = 0; c < cin; ++c) b[i * cin + c] = _Float16(a[int64_t(c) * nvox + i]);
}

__global__ void k_f32_to_f16(int64_t n, const float* a, _Float16* b) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        b[i] = _Float16(a[i]);
}

// W'[ci][t][co] = W[co][26 - t][ci] (backward-data weights)
__global__ void k_flip_weights(int cout, int cin, const _Float16* W, _Float16* Wt) {
    const int i = blockIdx.x * TPB + threadIdx.x;
    if (i >= cout * 27 * cin) return;
    const int co = i / (27 * cin), rem = i % (27 * cin), t = rem / cin, ci = rem % cin;
    Wt[(int64_t(ci) * 27 + (26 - t)) * cout + co] = W[i];
}

// Adam on FP32 masters: g = grad * gscale; updates w, m, v and the FP16 copy
__global__ void k_adam(int64_t n, float* w, float* m, float* v, const float* grad, _Float16* wh, float gscale,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        const float g = grad[i] * gscale;
        const float mi = b1 * m[i] + (1.f - b1) * g;
        const float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        wh[i] = _Float16(wi);
    }
}

// count of non-finite gradient entries (a half-precision overflow in the
// backward pass shows up here as inf or NaN)
__global__ void k_count_nonfinite(int64_t n, const float* g, int* count) {
    int c = 0;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        c += std::isfinite(g[i]) ? 0 : 1;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    __shared__ int sh[TPB / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) count[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_fill_f32(int64_t n, float* a, float val) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) a[i] = val;
}

int64_t gfor(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    return g < 1 ? 1 : (g > 4096 ? 4096 : g);
}

template <int CIN, int COUT, int MODE>
void conv_launch(const Geo& g, int dil, const _Float16* in, const _Float16* W, const _Float16* b,
                 const _Float16* mask, void* out, hipStream_t s) {
    const int64_t tiles = (g.nvox + 15) / 16;
    const int64_t blocks = (tiles + 3) / 4;
    hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), dim3(blocks), dim3(TPB), 0, s, g, dil, in, W, b, mask, out);
}

// nblk workgroups along the voxels, each writing one partial gradient
template <int CIN, int COUT>
void wgrad_launch(const Geo& g, int dil, const _Float16* in, const _Float16* dout, float* part, int nblk,
                  float* grad, hipStream_t s) {
    constexpr int NW = COUT * 27 * CIN + COUT;
    constexpr int TPW = CIN >= 32 ? 4 : 1;
    constexpr int NTN = (27 * CIN + 1 + 15) / 16;
    constexpr int groups = (NTN + 4 * TPW - 1) / (4 * TPW);
    hipLaunchKernelGGL((k_conv_wgrad<CIN, COUT, TPW>), dim3(nblk, groups), dim3(TPB), 0, s, g, dil, in, dout, part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3((NW + TPB - 1) / TPB), dim3(TPB), 0, s, part, nblk, NW, grad);
}

}  // namespace

// ---------------------------------------------------------------------------
// Net
// ---------------------------------------------------------------------------

Net::Net(Ctx* c, int channels, int in_channels, int n_layers, const int* dilations, const int grid[3])
    : ctx(c), C(channels), CI(in_channels), L(n_layers) {
    TBH_REQUIRE(channels == 32, "the surrogate kernels are built for 32 channels");
    TBH_REQUIRE(in_channels == 1 || in_channels == 4, "the surrogate kernels take 1 or 4 input channels");
    TBH_REQUIRE(n_layers >= 2 && n_layers <= MAX_LAYERS, "the surrogate takes 2 to 8 layers");
    for (int l = 0; l < L; ++l) {
        dil[l] = dilations ? dilations[l] : 1;
        TBH_REQUIRE(dil[l] >= 1 && dil[l] <= 64, "dilations must be in 1..64");
    }
    for (int a = 0; a < 3; ++a) {
        TBH_REQUIRE(grid[a] > 0, "grid sizes must be positive");
        g[a] = grid[a];
    }
    nvox = int64_t(g[0]) * g[1] * g[2];
    n_params = 0;
    for (int l = 0; l < L; ++l) {
        lin[l] = l == 0 ? CI : C;
        lout[l] = l == L - 1 ? 1 : C;
        off_w[l] = n_params;
        n_params += int64_t(lout[l]) * 27 * lin[l];
        off_b[l] = n_params;
        n_params += lout[l];
    }
    w32.alloc(n_params * 4);
    m32.alloc(n_params * 4);
    v32.alloc(n_params * 4);
    grad.alloc(n_params * 4);
    w16.alloc(n_params * 2);
    wt16.alloc(n_params * 2);
    for (int l = 0; l + 1 < L; ++l) act[l].alloc(size_t(nvox) * C * 2);   // hidden activations (FP16)
    xin.alloc(size_t(nvox) * CI * 2);
    pred.alloc(size_t(nvox) * 4);
    dact[0].alloc(size_t(nvox) * C * 2);
    dact[1].alloc(size_t(nvox) * C * 2);
    // workgroups of the weight gradient along the voxels (each 64-voxel chunk
    // belongs to one of them); one partial gradient each
    nchunk = int(std::min<int64_t>(256, std::max<int64_t>(1, (nvox + 63) / 64)));
    part.alloc(size_t(nchunk) * (int64_t(C) * 27 * C + C) * 4);
    dpart.alloc(4096 * 8);
    scalar.alloc(8 * 8);
    counts.alloc(64 * sizeof(int));
    step_t = 0;
    zero_moments();
}

void Net::set_loss_weights(const float* w_dev) {
    if (!w_dev) {
        weighted = false;
        return;
    }
    lw.alloc(size_t(nvox) * 4);
    TBH_HIP(hipMemcpyAsync(lw.p, w_dev, size_t(nvox) * 4, hipMemcpyDeviceToDevice, ctx->stream));
    weighted = true;
}

void Net::zero_moments() {
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_fill_f32, dim3(gfor(n_params)), dim3(TPB), 0, s, n_params, m32.as<float>(), 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(gfor(n_params)), dim3(TPB), 0, s, n_params, v32.as<float>(), 0.f);
    step_t = 0;
}

void Net::sync_half() {
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_f32_to_f16, dim3(gfor(n_params)), dim3(TPB), 0, s, n_params, w32.as<float>(),
                       w16.as<_Float16>());
    TBH_HIP(hipGetLastError());
}

void Net::forward(const float* x_dev, float* y_dev) {
    hipStream_t s = ctx->stream;
    const Geo geo{g[0], g[1], g[2], nvox};
    hipLaunchKernelGGL(k_pack_input, dim3(gfor(nvox)), dim3(TPB), 0, s, nvox, CI, x_dev, xin.as<_Float16>());
    const _Float16* W = w16.as<_Float16>();
    if (CI == 4)
        conv_launch<4, 32, 0>(geo, dil[0], xin.as<_Float16>(), W + off_w[0], W + off_b[0], nullptr, act[0].p, s);
    else
        conv_launch<1, 32, 0>(geo, dil[0], xin.as<_Float16>(), W + off_w[0], W + off_b[0], nullptr, act[0].p, s);
    for (int l = 1; l + 1 < L; ++l)
        conv_launch<32, 32, 0>(geo, dil[l], act[l - 1].as<_Float16>(), W + off_w[l], W + off_b[l], nullptr,
                               act[l].p, s);
    conv_launch<32, 1, 1>(geo, dil[L - 1], act[L - 2].as<_Float16>(), W + off_w[L - 1], W + off_b[L - 1], nullptr,
                          y_dev ? static_cast<void*>(y_dev) : pred.p, s);
    TBH_HIP(hipGetLastError());
}

double Net::accumulate_gradients(const float* x_dev, const float* t_dev) {
    hipStream_t s = ctx->stream;
    const Geo geo{g[0], g[1], g[2], nvox};
    forward(x_dev, nullptr);
    // loss gradient 2 w (pred - t) (weighted sum of squares), FP16, into dact[0] as [nvox][1]
    const int64_t gm = gfor(nvox);
    hipLaunchKernelGGL(k_mse, dim3(gm), dim3(TPB), 0, s, nvox, pred.as<float>(), t_dev,
                       weighted ? lw.as<float>() : static_cast<const float*>(nullptr), dact[0].as<_Float16>(),
                       dpart.as<double>());
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, s, dpart.as<double>(), int(gm), scalar.as<double>());
    const _Float16* W = w16.as<_Float16>();
    _Float16* Wt = wt16.as<_Float16>();
    float* gr = grad.as<float>();
    float* pt = part.as<float>();
    // from the last layer down: weight gradients from the layer's input and
    // upstream gradient, then backward-data through the layer into the
    // gradient of its input activations (ReLU mask of that input applied)
    int cur = 0;
    for (int l = L - 1; l >= 1; --l) {
        const _Float16* in = act[l - 1].as<_Float16>();
        const _Float16* up = dact[cur].as<_Float16>();
        _Float16* down = dact[1 - cur].as<_Float16>();
        const int nw = lout[l] * 27 * lin[l];
        hipLaunchKernelGGL(k_flip_weights, dim3((nw + TPB - 1) / TPB), dim3(TPB), 0, s, lout[l], lin[l],
                           W + off_w[l], Wt + off_w[l]);
        if (l == L - 1) {
            wgrad_launch<32, 1>(geo, dil[l], in, up, pt, nchunk, gr + off_w[l], s);
            conv_launch<1, 32, 2>(geo, dil[l], up, Wt + off_w[l], nullptr, in, down, s);
        } else {
            wgrad_launch<32, 32>(geo, dil[l], in, up, pt, nchunk, gr + off_w[l], s);
            conv_launch<32, 32, 2>(geo, dil[l], up, Wt + off_w[l], nullptr, in, down, s);
        }
        cur = 1 - cur;
    }
    // layer 0: weight gradients only
    if (CI == 4)
        wgrad_launch<4, 32>(geo, dil[0], xin.as<_Float16>(), dact[cur].as<_Float16>(), pt, nchunk, gr + off_w[0], s);
    else
        wgrad_launch<1, 32>(geo, dil[0], xin.as<_Float16>(), dact[cur].as<_Float16>(), pt, nchunk, gr + off_w[0], s);
    TBH_HIP(hipGetLastError());
    double loss = 0.0;
    TBH_HIP(hipMemcpyAsync(&loss, scalar.p, 8, hipMemcpyDeviceToHost, s));
    TBH_HIP(hipStreamSynchronize(s));
    return loss / double(nvox);
}

void Net::zero_grad() {
    hipLaunchKernelGGL(k_fill_f32, dim3(gfor(n_params)), dim3(TPB), 0, ctx->stream, n_params, grad.as<float>(), 0.f);
}

bool Net::adam(double lr, int batch) {
    // a step with a non-finite gradient entry is skipped: weights and moments
    // stay as they are
    const int64_t gb = std::min<int64_t>(gfor(n_params), 64);
    hipLaunchKernelGGL(k_count_nonfinite, dim3(gb), dim3(TPB), 0, ctx->stream, n_params, grad.as<float>(),
                       counts.as<int>());
    std::vector<int> cnt(static_cast<size_t>(gb));
    TBH_HIP(hipMemcpyAsync(cnt.data(), counts.p, size_t(gb) * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    TBH_HIP(hipStreamSynchronize(ctx->stream));
    for (int c : cnt)
        if (c != 0) return false;
    ++step_t;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, float(step_t)), c2 = 1.f - std::pow(b2, float(step_t));
    // gradient of the mean over voxels and samples
    const float gscale = float(1.0 / (double(nvox) * batch));
    hipLaunchKernelGGL(k_adam, dim3(gfor(n_params)), dim3(TPB), 0, ctx->stream, n_params, w32.as<float>(),
                       m32.as<float>(), v32.as<float>(), grad.as<float>(), w16.as<_Float16>(), gscale, float(lr),
                       b1, b2, eps, c1, c2);
    TBH_HIP(hipGetLastError());
    return true;
}

}  // namespace tbh
