// Block H.x for gfx950: y = D_i x_i + sum_b B_ib x_nbr(i,b) (+ U_i x_i).
//
// The Hamiltonian is the nearest-neighbour tight-binding matrix of the
// paper (Abstract; Sec. I); its application to a vector is the unit of cost
// of every Lanczos iteration the paper benchmarks (Sec. II-B).  On one GPU
// the operation is HBM-bound (about 0.5 flop per byte), so the kernel is
// organised around streaming the packed blocks once at full bandwidth:
//
//  * one 64-lane wavefront per tile of atoms; each lane owns R rows of one
//    atom and streams its private, chunk-interleaved segment of the block
//    array with 16-byte non-temporal loads (every wavefront load is one
//    contiguous L*16-byte read);
//  * neighbour vector slices are gathered through the cache hierarchy (the
//    whole x of a million-atom problem, 42 MB in FP32, stays in the 256 MB
//    Infinity Cache, and neighbouring atoms share lines in L2);
//  * workgroups are mapped XCD-contiguously, so the tiles one XCD processes
//    are spatial neighbours and share their gathered x lines in that XCD's L2;
//  * the Lanczos epilogue fuses y -= beta * x_prev and the FP64 partial sums
//    of Re(x^H y) and |y|^2 (wavefront shuffles, one partial pair per
//    wavefront; no atomics, fixed order).
#include "tbh_internal.h"

namespace tbh {

namespace {

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblk) {
    const int64_t xcd = bid % 8, idx = bid / 8, q = nblk / 8, r = nblk % 8;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Load n contiguous scalars starting at p (element offset off) with the
// widest aligned vector the static row size allows.
template <typename T, int N, int ROWBYTES>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&out)[N]) {
    if constexpr (ROWBYTES % 16 == 0 && (N * sizeof(T)) % 16 == 0) {
        typedef typename Vec16<T>::type V;
        constexpr int K = 16 / sizeof(T);
#pragma unroll
        for (int c = 0; c < N / K; ++c) {
            V v = reinterpret_cast<const V*>(p)[c];
#pragma unroll
            for (int e = 0; e < K; ++e) out[c * K + e] = v[e];
        }
    } else if constexpr (sizeof(T) == 4 && ROWBYTES % 8 == 0 && N % 2 == 0) {
        typedef float V2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int c = 0; c < N / 2; ++c) {
            V2 v = reinterpret_cast<const V2*>(p)[c];
            out[2 * c] = v[0];
            out[2 * c + 1] = v[1];
        }
    } else {
#pragma unroll
        for (int c = 0; c < N; ++c) out[c] = p[c];
    }
}

template <typename T, int N, int ROWBYTES>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&in)[N]) {
    if constexpr (ROWBYTES % 16 == 0 && (N * sizeof(T)) % 16 == 0) {
        typedef typename Vec16<T>::type V;
        constexpr int K = 16 / sizeof(T);
#pragma unroll
        for (int c = 0; c < N / K; ++c) {
            V v;
#pragma unroll
            for (int e = 0; e < K; ++e) v[e] = in[c * K + e];
            reinterpret_cast<V*>(p)[c] = v;
        }
    } else if constexpr (sizeof(T) == 4 && ROWBYTES % 8 == 0 && N % 2 == 0) {
        typedef float V2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int c = 0; c < N / 2; ++c) {
            V2 v;
            v[0] = in[2 * c];
            v[1] = in[2 * c + 1];
            reinterpret_cast<V2*>(p)[c] = v;
        }
    } else {
#pragma unroll
        for (int c = 0; c < N; ++c) p[c] = in[c];
    }
}

// acc[R rows] += M[R x NO] * xv[NO] where M is streamed chunk by chunk from
// the lane's segment (CH chunks of K scalars, row-major, padded at the end).
template <typename T, bool CPLX, int NO, int R>
__device__ __forceinline__ void stream_rows(const typename Vec16<T>::type* __restrict__ src, int L,
                                            const T (&xv)[NO * (CPLX ? 2 : 1)],
                                            T (&acc)[R * (CPLX ? 2 : 1)]) {
    constexpr int CS = CPLX ? 2 : 1;
    constexpr int K = 16 / sizeof(T);
    constexpr int S = R * NO * CS;
    constexpr int CH = (S + K - 1) / K;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const typename Vec16<T>::type v = __builtin_nontemporal_load(src + c * L);
        if constexpr (CPLX) {
#pragma unroll
            for (int e = 0; e < K; e += 2) {
                const int s = c * K + e;
                if (s < S) {
                    const int el = s / 2, r = el / NO, col = el % NO;
                    const T br = v[e], bi = v[e + 1];
                    const T xr = xv[2 * col], xi = xv[2 * col + 1];
                    acc[2 * r] = fma(br, xr, acc[2 * r]);
                    acc[2 * r] = fma(-bi, xi, acc[2 * r]);
                    acc[2 * r + 1] = fma(br, xi, acc[2 * r + 1]);
                    acc[2 * r + 1] = fma(bi, xr, acc[2 * r + 1]);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < K; ++e) {
                const int s = c * K + e;
                if (s < S) {
                    const int r = s / NO, col = s % NO;
                    acc[r] = fma(v[e], xv[col], acc[r]);
                }
            }
        }
    }
}

}  // namespace
}  // namespace tbh

#include <utility>
#include <algorithm>
namespace tbh { namespace {
template <typename T, bool CPLX, int NO, int R, bool DIAG, int C>
__device__ __forceinline__ void consume_chunk(const typename Vec16<T>::type& v, const T (&xv)[4][NO * (CPLX ? 2 : 1)],
                                              const T (&xo)[R * (CPLX ? 2 : 1)], const T (&xa)[DIAG ? 1 : NO * (CPLX ? 2 : 1)],
                                              T (&acc)[R * (CPLX ? 2 : 1)]) {
    constexpr int CS = CPLX ? 2 : 1;
    constexpr int K = 16 / sizeof(T);
    constexpr int S = R * NO * CS;
    constexpr int BC = (S + K - 1) / K;
    if constexpr (C < 4 * BC || !DIAG) {
        constexpr int seg = C / BC, cc = C % BC;
#pragma unroll
        for (int e = 0; e < K; e += CS) {
            const int s = cc * K + e;
            if (s < S) {
                if constexpr (CPLX) {
                    const int el = s / 2, r = el / NO, col = el % NO;
                    const T br = v[e], bi = v[e + 1];
                    T xr, xi;
                    if constexpr (seg < 4) { xr = xv[seg][2 * col]; xi = xv[seg][2 * col + 1]; }
                    else { xr = xa[2 * col]; xi = xa[2 * col + 1]; }
                    acc[2 * r] = fma(br, xr, acc[2 * r]);
                    acc[2 * r] = fma(-bi, xi, acc[2 * r]);
                    acc[2 * r + 1] = fma(br, xi, acc[2 * r + 1]);
                    acc[2 * r + 1] = fma(bi, xr, acc[2 * r + 1]);
                } else {
                    const int r = s / NO, col = s % NO;
                    T xval;
                    if constexpr (seg < 4) xval = xv[seg][col]; else xval = xa[col];
                    acc[r] = fma(v[e], xval, acc[r]);
                }
            }
        }
    } else {
        constexpr int cc = C - 4 * BC;
#pragma unroll
        for (int e = 0; e < K; ++e) {
            const int r = cc * K + e;
            if (r < R) {
#pragma unroll
                for (int q = 0; q < CS; ++q) acc[r * CS + q] = fma(v[e], xo[r * CS + q], acc[r * CS + q]);
            }
        }
    }
}
template <typename T, bool CPLX, int NO, int R, bool DIAG, int NCH, int D, int C>
__device__ __forceinline__ void pipe_step(const typename Vec16<T>::type* __restrict__ src, int L,
                                         typename Vec16<T>::type (&buf)[D], const T (&xv)[4][NO * (CPLX ? 2 : 1)],
                                         const T (&xo)[R * (CPLX ? 2 : 1)],
                                         const T (&xa)[DIAG ? 1 : NO * (CPLX ? 2 : 1)], T (&acc)[R * (CPLX ? 2 : 1)]) {
    const typename Vec16<T>::type v = buf[C % D];
    if constexpr (C + D < NCH) buf[C % D] = __builtin_nontemporal_load(src + (C + D) * L);
    consume_chunk<T, CPLX, NO, R, DIAG, C>(v, xv, xo, xa, acc);
}
template <typename T, bool CPLX, int NO, int R, bool DIAG, int NCH, int D, int... Cs>
__device__ __forceinline__ void pipe_all(std::integer_sequence<int, Cs...>, const typename Vec16<T>::type* __restrict__ src, int L,
                                         typename Vec16<T>::type (&buf)[D], const T (&xv)[4][NO * (CPLX ? 2 : 1)],
                                         const T (&xo)[R * (CPLX ? 2 : 1)],
                                         const T (&xa)[DIAG ? 1 : NO * (CPLX ? 2 : 1)], T (&acc)[R * (CPLX ? 2 : 1)]) {
    (pipe_step<T, CPLX, NO, R, DIAG, NCH, D, Cs>(src, L, buf, xv, xo, xa, acc), ...);
}
}}
namespace tbh {
namespace {
// block chunks in flight per lane in the ring-buffered stream, and the
// largest lane stream (in 16-byte chunks) that uses it
#ifndef HX_RING
#define HX_RING 12
#endif
// wavefronts (tiles) per workgroup; 1, 2 and 4 measured the same on the
// million-atom alloy (5.30-5.33 TB/s fused)
constexpr int HX_WPB = 4;
#ifndef HX_PIPE_MAX
#define HX_PIPE_MAX 128
#endif

struct HxK {
    const void* blocks;
    const int32_t* nbr;
    const void* x;
    void* y;
    const double* pot;
    const void* xprev;
    const double* beta;
    double* partial;
    int64_t n_atoms;
    int64_t n_tiles;
    const uint8_t* keys;   // tabulated layout: key records [n][8]
};

template <typename T, bool CPLX, int NO, int R, bool DIAG, bool LZ>
__global__ __launch_bounds__(64 * HX_WPB) void hx_kernel(HxK a) {
    constexpr int CS = CPLX ? 2 : 1;
    constexpr int G = NO / R, A = 64 / G, L = A * G;
    constexpr int K = 16 / sizeof(T);
    constexpr int BC = (R * NO * CS + K - 1) / K;
    constexpr int ROW = NO * CS;                     // scalars per atom row block
    constexpr int ROWB = ROW * sizeof(T);
    constexpr int OWN = R * CS;                      // scalars this lane owns
    typedef typename Vec16<T>::type V;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t tile = blk * HX_WPB + wave;
    const int64_t atom = tile * A + lane / G;
    const int g = lane % G;
    const bool active = tile < a.n_tiles && lane < L && atom < a.n_atoms;

    const T* __restrict__ x = static_cast<const T*>(a.x);
    T acc[OWN];
#pragma unroll
    for (int k = 0; k < OWN; ++k) acc[k] = T(0);
    double pa = 0.0, pw = 0.0;

    if (active) {
        const V* src = static_cast<const V*>(a.blocks) + (tile * (4 * BC + (DIAG ? (R + K - 1) / K : BC))) * L + lane;
        constexpr int NCH = 4 * BC + (DIAG ? (R + K - 1) / K : BC);
        T xo[OWN];
        load_row<T, OWN, (R * CS * sizeof(T)) % 16 == 0 && ROWB % 16 == 0 ? 16 : ((R * CS * sizeof(T)) % 8 == 0 && ROWB % 8 == 0 ? 8 : 4)>(
            x + atom * ROW + g * OWN, xo);
        if constexpr (NCH <= HX_PIPE_MAX) {
            // every gather first, then one ring-buffered stream of all block
            // chunks (loads complete in issue order, so x must be in flight
            // before the blocks for the stream's waits to stay shallow).  A
            // dangling slot reads the atom's own x against its all-zero block.
            T xv[4][ROW];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int32_t j = a.nbr[atom * 4 + b];
                load_row<T, ROW, ROWB>(x + (j >= 0 ? int64_t(j) : atom) * ROW, xv[b]);
            }
            T xa[DIAG ? 1 : ROW];
            if constexpr (!DIAG) load_row<T, ROW, ROWB>(x + atom * ROW, xa);
            constexpr int D = NCH < HX_RING ? NCH : HX_RING;
            V buf[D];
#pragma unroll
            for (int c = 0; c < D; ++c) buf[c] = __builtin_nontemporal_load(src + c * L);
            pipe_all<T, CPLX, NO, R, DIAG, NCH, D>(std::make_integer_sequence<int, NCH>{}, src, L, buf, xv, xo, xa, acc);
        } else {
            int32_t nb[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) nb[b] = a.nbr[atom * 4 + b];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (nb[b] >= 0) {
                    T xv[ROW];
                    load_row<T, ROW, ROWB>(x + int64_t(nb[b]) * ROW, xv);
                    stream_rows<T, CPLX, NO, R>(src + b * BC * L, L, xv, acc);
                }
            }
            const V* osrc = src + 4 * BC * L;
            if constexpr (DIAG) {
                constexpr int OC = (R + K - 1) / K;
#pragma unroll
                for (int c = 0; c < OC; ++c) {
                    const V v = __builtin_nontemporal_load(osrc + c * L);
#pragma unroll
                    for (int e = 0; e < K; ++e) {
                        const int r = c * K + e;
                        if (r < R) {
#pragma unroll
                            for (int q = 0; q < CS; ++q) acc[r * CS + q] = fma(v[e], xo[r * CS + q], acc[r * CS + q]);
                        }
                    }
                }
            } else {
                T xa[ROW];
                load_row<T, ROW, ROWB>(x + atom * ROW, xa);
                stream_rows<T, CPLX, NO, R>(osrc, L, xa, acc);
            }
        }
        if (a.pot) {
            const T u = T(a.pot[atom]);
#pragma unroll
            for (int k = 0; k < OWN; ++k) acc[k] = fma(u, xo[k], acc[k]);
        }
        if constexpr (LZ) {
            if (a.xprev) {
                const T bt = T(*a.beta);
                T xp[OWN];
                load_row<T, OWN, 4>(static_cast<const T*>(a.xprev) + atom * ROW + g * OWN, xp);
#pragma unroll
                for (int k = 0; k < OWN; ++k) acc[k] = fma(-bt, xp[k], acc[k]);
            }
#pragma unroll
            for (int k = 0; k < OWN; ++k) {
                pa += double(xo[k]) * double(acc[k]);
                pw += double(acc[k]) * double(acc[k]);
            }
        }
        store_row<T, OWN, (R * CS * sizeof(T)) % 16 == 0 && ROWB % 16 == 0 ? 16 : ((R * CS * sizeof(T)) % 8 == 0 && ROWB % 8 == 0 ? 8 : 4)>(
            static_cast<T*>(a.y) + atom * ROW + g * OWN, acc);
    }
    if constexpr (LZ) {
        // Re(x^H y) = sum over real scalars of x*y for interleaved complex;
        // one partial pair per wavefront (no workgroup barrier: a finished
        // wavefront does not wait for its siblings)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            pa += __shfl_xor(pa, off, 64);
            pw += __shfl_xor(pw, off, 64);
        }
        if (lane == 0 && a.partial) {
            const int64_t slot = int64_t(blockIdx.x) * HX_WPB + wave;
            a.partial[2 * slot] = pa;
            a.partial[2 * slot + 1] = pw;
        }
    }
}

template <typename T, bool CPLX, int NO, int R, bool DIAG>
void launch_one(const Layout& lay, const HxArgs& h, hipStream_t s) {
    HxK k{};
    k.blocks = h.blocks;
    k.nbr = h.nbr;
    k.x = h.x;
    k.y = h.y;
    k.pot = h.pot;
    k.xprev = h.xprev;
    k.beta = h.beta;
    k.partial = h.partial;
    k.n_atoms = h.n_atoms;
    k.n_tiles = lay.n_tiles;
    const int64_t nblk = (lay.n_tiles + HX_WPB - 1) / HX_WPB;
    if (nblk == 0) return;
    if (h.partial)
        hipLaunchKernelGGL((hx_kernel<T, CPLX, NO, R, DIAG, true>), dim3(nblk), dim3(64 * HX_WPB), 0, s, k);
    else
        hipLaunchKernelGGL((hx_kernel<T, CPLX, NO, R, DIAG, false>), dim3(nblk), dim3(64 * HX_WPB), 0, s, k);
}

template <typename T, bool CPLX, int NO, int R>
void launch_diag(const Layout& lay, const HxArgs& h, hipStream_t s) {
    if (lay.diag)
        launch_one<T, CPLX, NO, R, true>(lay, h, s);
    else
        launch_one<T, CPLX, NO, R, false>(lay, h, s);
}

template <typename T, bool CPLX>
void launch_shape(const Layout& lay, const HxArgs& h, hipStream_t s) {
    const int no = lay.n_o, r = lay.R;
#define TBH_CASE(NO_, R_)                                   \
    if (no == NO_ && r == R_) {                             \
        launch_diag<T, CPLX, NO_, R_>(lay, h, s);           \
        return;                                             \
    }
    TBH_CASE(5, 5)
    TBH_CASE(5, 1)
    TBH_CASE(10, 10)
    TBH_CASE(10, 5)
    TBH_CASE(10, 2)
    if constexpr (CPLX) {
        TBH_CASE(20, 20)
        TBH_CASE(20, 10)
        TBH_CASE(20, 4)
    }
#undef TBH_CASE
    throw Error(TBH_EINVAL, "no H.x kernel for n_o=" + std::to_string(no) + " rows/lane=" + std::to_string(r));
}


// ---------------------------------------------------------------------------
// Spin-diagonal bond blocks (H with spin at Gamma).  The two-centre hopping
// does not act on spin, so every bond block is I_2 (x) b with b real
// (NB x NB, NB = NO / 2); the spin-orbit term lives in the complex on-site
// block.  A lane owns R orbitals in both spins (2R complex rows of y); its
// stream holds, per bond, its R rows of b (R NB reals), then its 2R complex
// on-site rows (spin up rows, then spin down).  Per bond it reads R NB
// scalars instead of R NO complex ones (a quarter), and each b element
// multiplies the neighbour's x in both spins.
// ---------------------------------------------------------------------------
template <typename T, int NB, int R, int C>
__device__ __forceinline__ void consume_sd(const typename Vec16<T>::type& v, const T (&xv)[4][4 * NB],
                                           const T (&xa)[4 * NB], T (&acc)[4 * R]) {
    constexpr int NO = 2 * NB;
    constexpr int K = 16 / sizeof(T);
    constexpr int BC = (R * NB + K - 1) / K;
    if constexpr (C < 4 * BC) {
        constexpr int seg = C / BC, cc = C % BC;
#pragma unroll
        for (int e = 0; e < K; ++e) {
            const int s = cc * K + e;
            if (s < R * NB) {
                const int r = s / NB, c = s % NB;
                const T b = v[e];
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    acc[(sp * R + r) * 2] = fma(b, xv[seg][(sp * NB + c) * 2], acc[(sp * R + r) * 2]);
                    acc[(sp * R + r) * 2 + 1] = fma(b, xv[seg][(sp * NB + c) * 2 + 1], acc[(sp * R + r) * 2 + 1]);
                }
            }
        }
    } else {
        constexpr int cc = C - 4 * BC;
#pragma unroll
        for (int e = 0; e < K; e += 2) {
            const int s = cc * K + e;
            if (s < 2 * R * NO * 2) {
                const int el = s / 2, row = el / NO, col = el % NO;
                const T br = v[e], bi = v[e + 1];
                const T xr = xa[2 * col], xi = xa[2 * col + 1];
                acc[2 * row] = fma(br, xr, acc[2 * row]);
                acc[2 * row] = fma(-bi, xi, acc[2 * row]);
                acc[2 * row + 1] = fma(br, xi, acc[2 * row + 1]);
                acc[2 * row + 1] = fma(bi, xr, acc[2 * row + 1]);
            }
        }
    }
}

template <typename T, int NB, int R, int NCH, int D, int C>
__device__ __forceinline__ void sd_step(const typename Vec16<T>::type* __restrict__ src, int L,
                                        typename Vec16<T>::type (&buf)[D], const T (&xv)[4][4 * NB],
                                        const T (&xa)[4 * NB], T (&acc)[4 * R]) {
    const typename Vec16<T>::type v = buf[C % D];
    if constexpr (C + D < NCH) buf[C % D] = __builtin_nontemporal_load(src + (C + D) * L);
    consume_sd<T, NB, R, C>(v, xv, xa, acc);
}

template <typename T, int NB, int R, int NCH, int D, int... Cs>
__device__ __forceinline__ void sd_all(std::integer_sequence<int, Cs...>, const typename Vec16<T>::type* __restrict__ src,
                                       int L, typename Vec16<T>::type (&buf)[D], const T (&xv)[4][4 * NB],
                                       const T (&xa)[4 * NB], T (&acc)[4 * R]) {
    (sd_step<T, NB, R, NCH, D, Cs>(src, L, buf, xv, xa, acc), ...);
}

template <typename T, int NB, int R, bool LZ>
__global__ __launch_bounds__(64 * HX_WPB) void hx_sd_kernel(HxK a) {
    constexpr int NO = 2 * NB;
    constexpr int G = NB / R, A = 64 / G, L = A * G;
    constexpr int K = 16 / sizeof(T);
    constexpr int BC = (R * NB + K - 1) / K;
    constexpr int OC = (2 * R * NO * 2 + K - 1) / K;
    constexpr int NCH = 4 * BC + OC;
    constexpr int ROW = NO * 2;                      // scalars per atom row block
    constexpr int ROWB = ROW * int(sizeof(T));
    constexpr int HALF = 2 * R;                      // scalars of one spin's owned rows
    constexpr int HB = (HALF * int(sizeof(T))) % 16 == 0 ? 16 : ((HALF * int(sizeof(T))) % 8 == 0 ? 8 : 4);
    static_assert(NCH <= HX_PIPE_MAX, "lane stream too long for the ring-buffered pipeline");
    typedef typename Vec16<T>::type V;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t tile = blk * HX_WPB + wave;
    const int64_t atom = tile * A + lane / G;
    const int g = lane % G;
    const bool active = tile < a.n_tiles && lane < L && atom < a.n_atoms;

    const T* __restrict__ x = static_cast<const T*>(a.x);
    T acc[4 * R];
#pragma unroll
    for (int k = 0; k < 4 * R; ++k) acc[k] = T(0);
    double pa = 0.0, pw = 0.0;

    if (active) {
        const V* src = static_cast<const V*>(a.blocks) + tile * NCH * L + lane;
        // own rows: orbitals gR..gR+R-1 of spin up, then of spin down
        T xo[4 * R];
        {
            T h0[HALF], h1[HALF];
            load_row<T, HALF, HB>(x + atom * ROW + g * HALF, h0);
            load_row<T, HALF, HB>(x + atom * ROW + NB * 2 + g * HALF, h1);
#pragma unroll
            for (int k = 0; k < HALF; ++k) {
                xo[k] = h0[k];
                xo[HALF + k] = h1[k];
            }
        }
        T xv[4][ROW];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int32_t j = a.nbr[atom * 4 + b];
            load_row<T, ROW, ROWB>(x + (j >= 0 ? int64_t(j) : atom) * ROW, xv[b]);
        }
        T xa[ROW];
        load_row<T, ROW, ROWB>(x + atom * ROW, xa);
        constexpr int D = NCH < HX_RING ? NCH : HX_RING;
        V buf[D];
#pragma unroll
        for (int c = 0; c < D; ++c) buf[c] = __builtin_nontemporal_load(src + c * L);
        sd_all<T, NB, R, NCH, D>(std::make_integer_sequence<int, NCH>{}, src, L, buf, xv, xa, acc);
        if (a.pot) {
            const T u = T(a.pot[atom]);
#pragma unroll
            for (int k = 0; k < 4 * R; ++k) acc[k] = fma(u, xo[k], acc[k]);
        }
        if constexpr (LZ) {
            if (a.xprev) {
                const T bt = T(*a.beta);
                const T* xpv = static_cast<const T*>(a.xprev);
                T h0[HALF], h1[HALF];
                load_row<T, HALF, HB>(xpv + atom * ROW + g * HALF, h0);
                load_row<T, HALF, HB>(xpv + atom * ROW + NB * 2 + g * HALF, h1);
#pragma unroll
                for (int k = 0; k < HALF; ++k) {
                    acc[k] = fma(-bt, h0[k], acc[k]);
                    acc[HALF + k] = fma(-bt, h1[k], acc[HALF + k]);
                }
            }
#pragma unroll
            for (int k = 0; k < 4 * R; ++k) {
                pa += double(xo[k]) * double(acc[k]);
                pw += double(acc[k]) * double(acc[k]);
            }
        }
        T* y = static_cast<T*>(a.y) + atom * ROW;
        T h0[HALF], h1[HALF];
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            h0[k] = acc[k];
            h1[k] = acc[HALF + k];
        }
        store_row<T, HALF, HB>(y + g * HALF, h0);
        store_row<T, HALF, HB>(y + NB * 2 + g * HALF, h1);
    }
    if constexpr (LZ) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            pa += __shfl_xor(pa, off, 64);
            pw += __shfl_xor(pw, off, 64);
        }
        if (lane == 0 && a.partial) {
            const int64_t slot = int64_t(blockIdx.x) * HX_WPB + wave;
            a.partial[2 * slot] = pa;
            a.partial[2 * slot + 1] = pw;
        }
    }
}

template <typename T, int NB, int R>
void launch_sd(const Layout& lay, const HxArgs& h, hipStream_t s) {
    HxK k{};
    k.blocks = h.blocks;
    k.nbr = h.nbr;
    k.x = h.x;
    k.y = h.y;
    k.pot = h.pot;
    k.xprev = h.xprev;
    k.beta = h.beta;
    k.partial = h.partial;
    k.n_atoms = h.n_atoms;
    k.n_tiles = lay.n_tiles;
    const int64_t nblk = (lay.n_tiles + HX_WPB - 1) / HX_WPB;
    if (nblk == 0) return;
    if (h.partial)
        hipLaunchKernelGGL((hx_sd_kernel<T, NB, R, true>), dim3(nblk), dim3(64 * HX_WPB), 0, s, k);
    else
        hipLaunchKernelGGL((hx_sd_kernel<T, NB, R, false>), dim3(nblk), dim3(64 * HX_WPB), 0, s, k);
}

// ---------------------------------------------------------------------------
// Tabulated bond blocks.  In an unstrained real H at Gamma every bond block
// is fixed by (sublattice, species pair, bond slot): the two-centre
// Slater-Koster form depends only on the species and the bond direction.  The
// table of the distinct blocks (12.8 KB for a two-species sp3d5s* alloy in
// FP32) is staged in LDS once per workgroup; per atom the kernel streams an
// 8-byte key record, the neighbour indices and the vectors, about 110 bytes
// instead of 1.7 KB.  One atom per lane, one tile of 64 atoms per wavefront.
// ---------------------------------------------------------------------------
// LDS offset of table block `key`: 16 bytes of padding after every 8 blocks.
// The keys that one bond slot takes across a wavefront differ by multiples
// of 4 (the dense key order is sublattice, species, neighbour species,
// slot), so unpadded 100-element blocks put all of them on two bank groups;
// with the padding the 8 keys of a slot start on 8 different groups of 4
// banks and stay 16-byte aligned.
template <typename T, int NO>
__host__ __device__ constexpr int tab_block_offset(int key) {
    return key * NO * NO + (16 / int(sizeof(T))) * (key >> 3);
}

template <typename T, int NO, bool LZ>
__global__ __launch_bounds__(64 * HX_WPB) void hx_tab_kernel(HxK a, int nu, int ns) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* tab = reinterpret_cast<T*>(smem);
    constexpr int ROWB = NO * sizeof(T);
    constexpr int BB = NO * NO;
    const T* __restrict__ gt = static_cast<const T*>(a.blocks);
    for (int i = threadIdx.x; i < nu * BB; i += blockDim.x) tab[tab_block_offset<T, NO>(i / BB) + i % BB] = gt[i];
    const int d0 = tab_block_offset<T, NO>(nu);   // the on-site diagonals follow the last block
    for (int i = threadIdx.x; i < ns * NO; i += blockDim.x) tab[d0 + i] = gt[nu * BB + i];
    __syncthreads();

    // Each XCD owns a contiguous share of the units of HX_WPB tiles, in
    // proportion to its blocks, and its blocks sweep that share together
    // (grid-stride within the XCD): the table is staged once per resident
    // block while the units in flight on an XCD stay adjacent, so gathered
    // rows a cell plane back still hit its L2.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n_units = (a.n_tiles + HX_WPB - 1) / HX_WPB;
    const int64_t G = gridDim.x, xcd = blockIdx.x % 8, q = G / 8, rem = G % 8;
    const int64_t b_lo = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    const int64_t xcd_blocks = q + (xcd < rem ? 1 : 0);   // blocks of this XCD
    const int64_t u_lo = n_units * b_lo / G, u_hi = n_units * (b_lo + xcd_blocks) / G;
    const T* __restrict__ x = static_cast<const T*>(a.x);
    double pa = 0.0, pw = 0.0;
    for (int64_t u = u_lo + blockIdx.x / 8; u < u_hi; u += xcd_blocks) {
        const int64_t atom = (u * HX_WPB + wave) * 64 + lane;
        if (atom >= a.n_atoms) continue;
        const uint2 kr = reinterpret_cast<const uint2*>(a.keys)[atom];
        const int4 nb4 = reinterpret_cast<const int4*>(a.nbr)[atom];
        const int32_t nbs[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
        T xo[NO];
        load_row<T, NO, ROWB>(x + atom * NO, xo);
        T xv[4][NO];
#pragma unroll
        for (int b = 0; b < 4; ++b) load_row<T, NO, ROWB>(x + (nbs[b] >= 0 ? int64_t(nbs[b]) : atom) * NO, xv[b]);
        const int sp = int(kr.y & 0xffu);
        const T u_at = a.pot ? T(a.pot[atom]) : T(0);
        T acc[NO];
        const T* __restrict__ dg = tab + d0 + sp * NO;
#pragma unroll
        for (int r = 0; r < NO; ++r) acc[r] = (dg[r] + u_at) * xo[r];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const unsigned key = (kr.x >> (8 * b)) & 0xffu;
            if (key == 255u) continue;   // dangling bond
            const T* __restrict__ B = tab + tab_block_offset<T, NO>(int(key));
#pragma unroll
            for (int r = 0; r < NO; ++r)
#pragma unroll
                for (int c = 0; c < NO; ++c) acc[r] = fma(B[r * NO + c], xv[b][c], acc[r]);
        }
        if constexpr (LZ) {
            if (a.xprev) {
                const T bt = T(*a.beta);
                T xp[NO];
                load_row<T, NO, ROWB>(static_cast<const T*>(a.xprev) + atom * NO, xp);
#pragma unroll
                for (int k = 0; k < NO; ++k) acc[k] = fma(-bt, xp[k], acc[k]);
            }
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                pa += double(xo[k]) * double(acc[k]);
                pw += double(acc[k]) * double(acc[k]);
            }
        }
        store_row<T, NO, ROWB>(static_cast<T*>(a.y) + atom * NO, acc);
    }
    if constexpr (LZ) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            pa += __shfl_xor(pa, off, 64);
            pw += __shfl_xor(pw, off, 64);
        }
        if (lane == 0 && a.partial) {
            const int64_t slot = int64_t(blockIdx.x) * HX_WPB + wave;
            a.partial[2 * slot] = pa;
            a.partial[2 * slot + 1] = pw;
        }
    }
}

size_t tab_lds_bytes(const Layout& lay) {
    // the blocks with their padding (16 bytes per 8 blocks, as tab_block_offset), then the diagonals
    return (size_t(lay.nu) * lay.n_o * lay.n_o + size_t(lay.ns) * lay.n_o) * size_t(lay.esz) +
           16 * size_t(lay.nu >> 3);
}

template <typename T, int NO>
void launch_tab(const Layout& lay, const HxArgs& h, hipStream_t s) {
    HxK k{};
    k.blocks = h.blocks;
    k.nbr = h.nbr;
    k.x = h.x;
    k.y = h.y;
    k.pot = h.pot;
    k.xprev = h.xprev;
    k.beta = h.beta;
    k.partial = h.partial;
    k.n_atoms = h.n_atoms;
    k.n_tiles = lay.n_tiles;
    k.keys = h.keys;
    TBH_REQUIRE(h.keys, "tabulated layout without key records");
    if (lay.tab_grid == 0) return;
    TBH_REQUIRE(lay.tab_grid <= INT32_MAX, "tabulated launch too large");
    const size_t lds = tab_lds_bytes(lay);
    TBH_REQUIRE(lds <= 49152, "block table larger than 48 KB");
    const dim3 g(unsigned(lay.tab_grid)), blk(64 * HX_WPB);
    if (h.partial)
        hipLaunchKernelGGL((hx_tab_kernel<T, NO, true>), g, blk, lds, s, k, lay.nu, lay.ns);
    else
        hipLaunchKernelGGL((hx_tab_kernel<T, NO, false>), g, blk, lds, s, k, lay.nu, lay.ns);
}

// resident blocks of the fused (Lanczos) instance on the current device
template <typename T, int NO>
int tab_resident(size_t lds) {
    int dev = 0, cus = 0, occ = 0;
    TBH_HIP(hipGetDevice(&dev));
    TBH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TBH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, hx_tab_kernel<T, NO, true>, 64 * HX_WPB, lds));
    return std::max(1, cus * std::max(1, occ));
}

}  // namespace

bool hx_shape_supported(int n_o, bool cplx_h, int R) {
    if (n_o == 5) return R == 5 || R == 1;
    if (n_o == 10) return R == 10 || R == 5 || R == 2;
    if (n_o == 20) return cplx_h && (R == 20 || R == 10 || R == 4);
    return false;
}

// partial-sum slots a fused Lanczos launch writes (one per wavefront)
int64_t hx_num_blocks(const Layout& lay) {
    if (lay.tab) return HX_WPB * lay.tab_grid;
    return HX_WPB * ((lay.n_tiles + HX_WPB - 1) / HX_WPB);
}

void hx_tab_configure(Layout& lay) {
    TBH_REQUIRE(lay.tab && (lay.n_o == 5 || lay.n_o == 10), "tabulated blocks need 5 or 10 orbitals");
    const size_t lds = tab_lds_bytes(lay);
    int res;
    if (lay.esz == 8) res = lay.n_o == 5 ? tab_resident<double, 5>(lds) : tab_resident<double, 10>(lds);
    else res = lay.n_o == 5 ? tab_resident<float, 5>(lds) : tab_resident<float, 10>(lds);
    const int64_t n_units = (lay.n_tiles + HX_WPB - 1) / HX_WPB;
    lay.tab_grid = std::min<int64_t>(n_units, res);
}

void hx_launch(const Layout& lay, bool f64, const HxArgs& h, hipStream_t s) {
    if (lay.tab) {
        TBH_REQUIRE(lay.n_o == 5 || lay.n_o == 10, "tabulated blocks need 5 or 10 orbitals");
        if (f64) {
            if (lay.n_o == 5) launch_tab<double, 5>(lay, h, s);
            else launch_tab<double, 10>(lay, h, s);
        } else {
            if (lay.n_o == 5) launch_tab<float, 5>(lay, h, s);
            else launch_tab<float, 10>(lay, h, s);
        }
        TBH_HIP(hipGetLastError());
        return;
    }
    if (lay.sd) {
        TBH_REQUIRE((lay.n_o == 20 && lay.R == 2) || (lay.n_o == 10 && lay.R == 1),
                    "spin-diagonal blocks: 20 orbitals with 2 rows per lane or 10 with 1");
        if (lay.n_o == 20) {
            if (f64) launch_sd<double, 10, 2>(lay, h, s);
            else launch_sd<float, 10, 2>(lay, h, s);
        } else {
            if (f64) launch_sd<double, 5, 1>(lay, h, s);
            else launch_sd<float, 5, 1>(lay, h, s);
        }
        TBH_HIP(hipGetLastError());
        return;
    }
    const bool c = lay.cs == 2;
    if (f64) {
        if (c) launch_shape<double, true>(lay, h, s);
        else launch_shape<double, false>(lay, h, s);
    } else {
        if (c) launch_shape<float, true>(lay, h, s);
        else launch_shape<float, false>(lay, h, s);
    }
    TBH_HIP(hipGetLastError());
}

}  // namespace tbh
