// Multi-vector H.X on the matrix cores, single Hamiltonian or a batch of
// many (cells x k-points) in one persistent launch.
//
// The paper groups independent k-points (and biases) into separate solver
// groups (Sec. II-C, multi-level parallelism, Fig. 1b).  On one GPU the
// groups become one launch over the concatenated atoms of every
// (cell, k-point) Hamiltonian, and several right-hand vectors per atom turn
// every block product into a small dense GEMM:
//
//   Y_i (n_o x R) = [B_i0 B_i1 B_i2 B_i3 D_i] [X_n0; X_n1; X_n2; X_n3; X_i]
//
// Complex blocks are handled with the real embedding
//   [Yr; Yi] = [[Br, -Bi], [Bi, Br]] [Xr; Xi],
// computed as Y^T = X^T A^T with v_mfma_f32_16x16x4f32: the right-hand
// vectors are the 16-wide M dimension, the embedded output rows the N
// dimension (two 16-wide tiles for 20 rows), K = 5 n_o (x2 for complex).
// One wavefront owns one atom at a time: it stages the atom's five blocks
// (4 KB for 10x10 complex) into LDS, reads its B-operand from LDS and
// gathers the X rows of the neighbours straight from L2, every gather of the
// atom in flight at once.  The next atom's blocks and neighbour indices are
// loaded into registers (16-byte non-temporal loads) while the current
// atom's products run.
// A persistent grid walks the concatenated atom range: either one window of
// consecutive atoms for the whole grid (each XCD a contiguous part of it), or
// one contiguous share per XCD swept by that XCD's workgroups, so that one
// XCD's L2 holds the X rows its neighbouring atoms share.
#include "tbh_internal.h"
#include "hx_multi.h"

namespace tbh {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblk, int remap) {
    if (!remap) return bid;
    const int64_t xcd = bid % 8, idx = bid / 8, q = nblk / 8, r = nblk % 8;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <bool CPLX, int NO, int NRHS>
__global__ __launch_bounds__(64) void k_hx_mv(const MvDesc* __restrict__ desc, int n_inst, int64_t total,
                                              int remap) {
    constexpr int CS = CPLX ? 2 : 1;
    constexpr int ME = NO * CS;                 // embedded output rows
    constexpr int KE = 5 * NO * CS;             // embedded K
    constexpr int NT = (ME + 15) / 16;          // N tiles
    constexpr int KS = (KE + 3) / 4;            // K steps
    constexpr int MT = NRHS / 16;               // M tiles (right-hand vectors)
    constexpr int BF = 5 * NO * NO * CS;        // block floats per atom
    constexpr int BFP = (BF + 3) & ~3;          // padded to 16 bytes
    constexpr int NV = BFP / 4;                 // 16-byte chunks per atom
    constexpr int PV = (NV + 63) / 64;          // chunks per lane
    constexpr int DIAG0 = 4 * NO * NO * CS;     // first on-site float
    __shared__ float blk[BFP];

    const int lane = threadIdx.x;
    // the table may be a slice of a larger batch: its atom range starts at
    // desc[0].atom_begin and spans `total` atoms
    const int64_t base = desc[0].atom_begin;
    int64_t g, step, g_end;
    if (remap == 2 && gridDim.x >= 8) {
        // each XCD (workgroups are dispatched to the 8 XCDs round-robin) owns
        // one contiguous eighth of the atoms and its workgroups sweep it in
        // grid-stride order: successive windows on one XCD are neighbours,
        // so the X rows one window's halo needs are the next window's own
        // rows and stay in that XCD's L2
        const int xcd = int(blockIdx.x % 8);
        const int64_t idx = blockIdx.x / 8;
        step = (int64_t(gridDim.x) - xcd + 7) / 8;
        g = base + total * xcd / 8 + idx;
        g_end = base + total * (xcd + 1) / 8;
    } else {
        // grid-stride walk: at any moment the wavefronts in flight hold one
        // window of `gridDim.x` consecutive atoms (each XCD a contiguous part
        // of it with remap 1)
        step = gridDim.x;
        g = base + xcd_block(blockIdx.x, gridDim.x, remap);
        g_end = base + total;
    }
    if (g >= g_end) return;
    // instance containing g
    int inst = 0;
    while (inst + 1 < n_inst && desc[inst + 1].atom_begin <= g) ++inst;

    // software pipeline: the next atom's blocks and neighbour indices are
    // loaded into registers while the current atom's products run
    v4f pre[PV];
    int32_t pnb[4];
    auto prefetch = [&](int ins, int64_t gg) {
        const MvDesc& d = desc[ins];
        const int64_t at = gg - d.atom_begin;
        const v4f* src = reinterpret_cast<const v4f*>(d.blocks + at * BFP);
#pragma unroll
        for (int p = 0; p < PV; ++p) {
            const int c = lane + p * 64;
            if (c < NV) pre[p] = __builtin_nontemporal_load(src + c);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) pnb[s] = d.nbr[at * 4 + s];
    };
    prefetch(inst, g);

    for (; g < g_end; g += step) {
        const MvDesc& d = desc[inst];
        const int64_t atom = g - d.atom_begin;
        // stage the prefetched blocks (bonds 0..3, on-site + potential on its
        // diagonal) into LDS
        const float u = float((d.pot ? d.pot[atom] : 0.0) + d.shift);
#pragma unroll
        for (int p = 0; p < PV; ++p) {
            const int c = lane + p * 64;
            if (c < NV) {
                v4f v = pre[p];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int f = c * 4 + e - DIAG0;                 // on-site float index
                    if (f >= 0 && f < NO * NO * CS && (f / CS) % (NO + 1) == 0 && f % CS == 0) v[e] += u;
                }
                reinterpret_cast<v4f*>(blk)[c] = v;
            }
        }
        // neighbour rows of X (wave-uniform: one atom per wavefront)
        const float* __restrict__ X = d.x;
        const float* xb[5];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int32_t j = __builtin_amdgcn_readfirstlane(pnb[s]);
            xb[s] = X + (j >= 0 ? int64_t(j) : atom) * (NO * NRHS * CS);   // dangling: the block is zero
        }
        xb[4] = X + atom * (NO * NRHS * CS);
        __syncthreads();
        // the right-hand-side gathers of this atom, all in flight at once
        const int kl = lane >> 4, col = lane & 15;
        float a[KS][MT];
        if constexpr (CPLX && NO % 2 == 0) {
            // k = 4 ks + kl: part p = kl & 1, column c = 2 ks % NO + kl / 2,
            // slot s = 2 ks / NO (the same for all lanes since NO is even)
            const int lane_off = ((kl >> 1) * NRHS + col) * 2 + (kl & 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int s = (2 * ks) / NO, c0 = (2 * ks) % NO;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a[ks][mt] = xb[s][lane_off + (c0 * NRHS + mt * 16) * 2];
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = ks * 4 + kl;
                const int kk = k < KE ? k : 0;
                const int p = CPLX ? (kk & 1) : 0;
                const int sc = CPLX ? (kk >> 1) : kk;
                const int s = sc / NO, c = sc % NO;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    a[ks][mt] = k < KE ? xb[s][((c * NRHS) + mt * 16 + col) * CS + p] : 0.f;
            }
        }
        // next atom's blocks
        if (g + step < g_end) {
            int ins = inst;
            while (g + step >= desc[ins].atom_begin + desc[ins].n_atoms) ++ins;
            prefetch(ins, g + step);
        }
        v4f acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[mt][t] = v4f{0.f, 0.f, 0.f, 0.f};
        if constexpr (CPLX && NO % 2 == 0) {
            // B operand of output row m = 16 t + col, K index k = 4 ks + kl:
            // block float ((s NO + r) NO + c) 2 + q with s = 2 ks / NO,
            // c = 2 ks % NO + kl / 2 and a row part r, part q and sign fixed
            // per lane and tile, so every read is one lane base plus a
            // constant offset
            const int p = kl & 1, hh = kl >> 1;
            int bofs[NT];
            float sgn[NT];
            bool ok[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int m = t * 16 + col;
                ok[t] = m < ME;
                const int r = m < NO ? m : m - NO;
                const int q = m < NO ? p : 1 - p;
                sgn[t] = (m < NO && p == 1) ? -1.f : 1.f;
                bofs[t] = ok[t] ? 2 * (r * NO + hh) + q : 0;
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int s = (2 * ks) / NO, c0 = (2 * ks) % NO;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const float v = blk[bofs[t] + 2 * (s * NO * NO + c0)];
                    const float b = ok[t] ? sgn[t] * v : 0.f;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks][mt], b, acc[mt][t], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = ks * 4 + kl;
                const int kk = k < KE ? k : 0;
                const int p = CPLX ? (kk & 1) : 0;
                const int sc = CPLX ? (kk >> 1) : kk;
                const int s = sc / NO, c = sc % NO;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int m = t * 16 + col;
                    float b = 0.f;
                    if (k < KE && m < ME) {
                        if constexpr (CPLX) {
                            const int r = m < NO ? m : m - NO;
                            const int q = m < NO ? p : 1 - p;
                            const float v = blk[((s * NO + r) * NO + c) * 2 + q];
                            b = (m < NO && p == 1) ? -v : v;
                        } else {
                            b = blk[(s * NO + m) * NO + c];
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks][mt], b, acc[mt][t], 0, 0, 0);
                }
            }
        }
        // D[i = 4*(lane/16) + v][j = lane%16] = Y^T[rhs][m]
        float* __restrict__ Y = d.y;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int m = t * 16 + col;
                if (m < ME) {
                    const int r = CPLX ? (m < NO ? m : m - NO) : m;
                    const int p = CPLX ? (m < NO ? 0 : 1) : 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rhs = mt * 16 + 4 * kl + v;
                        Y[((atom * NO + r) * NRHS + rhs) * CS + p] = acc[mt][t][v];
                    }
                }
            }
        // every lane's LDS reads are done before the next atom overwrites blk
        __syncthreads();
        while (g + step < g_end && g + step >= desc[inst].atom_begin + desc[inst].n_atoms) ++inst;
    }
}

template <bool CPLX, int NO>
void launch_no(int nrhs, const MvDesc* desc, int n_inst, int64_t total, int grid, int remap, hipStream_t s) {
    if (nrhs == 16)
        hipLaunchKernelGGL((k_hx_mv<CPLX, NO, 16>), dim3(grid), dim3(64), 0, s, desc, n_inst, total, remap);
    else if (nrhs == 32)
        hipLaunchKernelGGL((k_hx_mv<CPLX, NO, 32>), dim3(grid), dim3(64), 0, s, desc, n_inst, total, remap);
    else if constexpr (!CPLX)
        if (nrhs == 64)
            hipLaunchKernelGGL((k_hx_mv<CPLX, NO, 64>), dim3(grid), dim3(64), 0, s, desc, n_inst, total, remap);
        else
            throw Error(TBH_EINVAL, "multi-vector H.X supports nrhs = 16, 32 (or 64 for a real H)");
    else
        throw Error(TBH_EINVAL, "multi-vector H.X supports nrhs = 16 or 32 for a complex H");
}

}  // namespace

bool mv_supported(int n_o, int nrhs) { return (n_o == 5 || n_o == 10 || n_o == 20) && (nrhs == 16 || nrhs == 32); }

int64_t mv_block_floats(int n_o, bool cplx_h) {
    const int64_t f = 5 * int64_t(n_o) * n_o * (cplx_h ? 2 : 1);
    return (f + 3) & ~int64_t(3);
}

void mv_launch(bool cplx_h, int n_o, int nrhs, const MvDesc* desc_dev, int n_inst, int64_t total_atoms, int grid,
               int remap, hipStream_t s) {
    if (total_atoms == 0) return;
    if (grid < 1) grid = 1;
    if (cplx_h) {
        if (n_o == 5) launch_no<true, 5>(nrhs, desc_dev, n_inst, total_atoms, grid, remap, s);
        else if (n_o == 10) launch_no<true, 10>(nrhs, desc_dev, n_inst, total_atoms, grid, remap, s);
        else if (n_o == 20) launch_no<true, 20>(nrhs, desc_dev, n_inst, total_atoms, grid, remap, s);
        else throw Error(TBH_EINVAL, "unsupported orbital count");
    } else {
        if (n_o == 5) launch_no<false, 5>(nrhs, desc_dev, n_inst, total_atoms, grid, remap, s);
        else if (n_o == 10) launch_no<false, 10>(nrhs, desc_dev, n_inst, total_atoms, grid, remap, s);
        else throw Error(TBH_EINVAL, "unsupported orbital count");
    }
    TBH_HIP(hipGetLastError());
}

}  // namespace tbh
