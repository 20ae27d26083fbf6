// Multi-vector H.X internals shared by hx_multi.hip and the C ABI.
#pragma once

#include "tbh_internal.h"

namespace tbh {

// one Hamiltonian of a batch (device-resident table entry)
struct MvDesc {
    const float* blocks;    // [n_atoms][5][n_o][n_o] (complex interleaved), per atom padded to 16 B
    const int32_t* nbr;     // [n_atoms][4]
    const double* pot;      // [n_atoms] or null
    const float* x;         // [n_atoms][n_o][nrhs] (complex interleaved)
    float* y;
    int64_t atom_begin;     // offset of this instance in the concatenated atom range
    int64_t n_atoms;
    double shift = 0.0;     // added to every diagonal element: Y = (H + shift) X
};

bool mv_supported(int n_o, int nrhs);
int64_t mv_block_floats(int n_o, bool cplx_h);
// y = H x for every instance; grid = persistent workgroups (one wavefront each)
void mv_launch(bool cplx_h, int n_o, int nrhs, const MvDesc* desc_dev, int n_inst, int64_t total_atoms, int grid,
               int remap, hipStream_t s);

}  // namespace tbh
