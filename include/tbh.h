/*
 * tbh.h -- C ABI of the MI355X tight-binding H.x / Lanczos / Schrodinger-Poisson
 * library (libtbh.so).
 *
 * The method is the one of Lee, Ryu, Jiang and Klimeck, "Million Atom
 * Electronic Structure and Device Calculations on Peta-Scale Computers":
 * an empirical sp3s* / sp3d5s* nearest-neighbour tight-binding Hamiltonian
 * with strain (Abstract; Sec. I), whose eigenstates near the band gap are
 * found with a Lanczos solver (Sec. III-A, item 1; the benchmark unit of
 * Sec. II-B is a fixed number of Lanczos iterations), inside a
 * self-consistent Schrodinger-Poisson loop (Sec. III-A).
 *
 * Conventions (all entry points):
 *  - Every call returns a status code (TBH_OK = 0 or a negative TBH_E*);
 *    nothing throws across the ABI.  tbh_last_error() returns a
 *    thread-local message for the last failing call on this thread.
 *  - On failure, outputs are left untouched unless the entry point says
 *    otherwise (TBH_ENOCONV writes partial results).
 *  - Pointers documented as "device" are HIP device pointers owned by the
 *    caller (the library never frees caller memory).  Pointers documented as
 *    "host" are ordinary host memory, read (or written) during the call only.
 *  - Objects (tbh_ctx, tbh_ham, ...) own their internal device storage and
 *    release it in the matching *_destroy call.
 *  - All device work is enqueued on the context's HIP stream.  Calls that
 *    return host values synchronise that stream before returning.
 *  - Complex vectors and blocks are interleaved (re, im) pairs.
 *  - Vector rows are atom-major, orbital-minor; with spin, the orbitals of
 *    one atom are spin-major: row = atom*n_o + spin*n_base + orbital.
 *  - Orbital order: sp3s* = [s, px, py, pz, s*];
 *    sp3d5s* = [s, px, py, pz, dxy, dyz, dzx, dx2-y2, d3z2-r2, s*].
 *  - Same inputs on the same GPU give bitwise identical outputs (all
 *    reductions are fixed-order; no floating-point atomics).
 *  - One context per host thread.
 */
#ifndef TBH_H
#define TBH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TBH_OK        0
#define TBH_EINVAL   -1   /* invalid argument (null pointer, bad size, bad geometry) */
#define TBH_ENOMEM   -2   /* device or host allocation failed */
#define TBH_EHIP     -3   /* a HIP runtime call failed */
#define TBH_ENOCONV  -4   /* an iteration did not converge; partial results written */
#define TBH_ESTATE   -5   /* object used in a wrong state */

/* tight-binding models (Abstract; Sec. I) */
#define TBH_SP3S     0    /* s, p(3), s*: 5 orbitals per atom and spin */
#define TBH_SP3D5S   1    /* s, p(3), d(5), s*: 10 orbitals per atom and spin */

/* storage precision of H and of the vectors it is applied to */
#define TBH_F64      0
#define TBH_F32      1

typedef struct tbh_ctx tbh_ctx;
typedef struct tbh_ham tbh_ham;

/* Library version (major*10000 + minor*100 + patch). */
int tbh_version(void);

/* Thread-local message of the last failing call; valid until the next call
 * on this thread.  Never NULL. */
const char* tbh_last_error(void);

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream must stay
 * valid until tbh_ctx_destroy. */
int tbh_ctx_create(int device, void* hip_stream, tbh_ctx** out);
int tbh_ctx_destroy(tbh_ctx* ctx);
/* Change the stream later calls enqueue on. */
int tbh_ctx_set_stream(tbh_ctx* ctx, void* hip_stream);

/* ------------------------------------------------------------------------
 * Geometry and parameters (host memory, copied during the build call).
 *
 * Atoms sit on the diamond lattice in integer coordinates of a/4:
 * sublattice A has all coordinates even with x+y+z = 0 (mod 4), sublattice
 * B = A + (1,1,1).  Every coordinate must satisfy 0 <= q < box_q on every
 * axis.  Bond slot b of an A atom points along d_b, with
 * d_0=(1,1,1), d_1=(1,-1,-1), d_2=(-1,1,-1), d_3=(-1,-1,1); slot b of a B
 * atom points along -d_b, so j = nbr(i,b) implies nbr(j,b) = i.  Periodic
 * axes wrap modulo box_q; on hard-wall axes a bond leaving the box is
 * dangling.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_atoms;
    const int32_t* pos_q;     /* host [n_atoms][3], a/4 units */
    const uint8_t* species;   /* host [n_atoms], each < n_species */
    int32_t box_q[3];         /* box edge per axis, a/4 units (4 * cells) */
    int32_t periodic[3];      /* 1 = periodic, 0 = hard wall */
} tbh_geometry;

/* Empirical tight-binding parameters (eV).
 * onsite[s] = (E_s, E_p, E_d, E_s*) of species s (E_d unused for sp3s*).
 * sk[a][b][14] = two-centre integrals of a bond between species a and b in
 * the order ss_sigma, s*s*_sigma, ss*_sigma, sp_sigma, s*p_sigma, sd_sigma,
 * s*d_sigma, pp_sigma, pp_pi, pd_sigma, pd_pi, dd_sigma, dd_pi, dd_delta
 * (Slater & Koster two-centre form; the d-shell ones unused for sp3s*).
 * The set must be symmetric (sk[a][b] == sk[b][a]).
 * so_delta[s] = spin-orbit splitting Delta of the p shell, used when spin=1:
 * on-site lambda L.S with lambda = 2 Delta / 3 (NULL = 0).
 * passivation_eV: each dangling bond adds passivation_eV * |h><h| to the
 * on-site block, h = (s + d.p)/2 the sp3 hybrid along the missing bond
 * (0 = off). */
typedef struct {
    int32_t model;            /* TBH_SP3S or TBH_SP3D5S */
    int32_t spin;             /* 0: no spin; 1: spin-major doubling + spin-orbit */
    int32_t n_species;        /* 1..16 */
    const double* onsite;     /* host [n_species][4] */
    const double* sk;         /* host [n_species][n_species][14] */
    const double* so_delta;   /* host [n_species] or NULL */
    double passivation_eV;
} tbh_params;

typedef struct {
    /* host [n_atoms][4] hopping scale per bond slot (strain), or NULL = 1.
     * Only rows of A-sublattice atoms are read; the reverse direction of a
     * bond uses its A atom's factor. */
    const double* bond_scale;
    /* host [n_atoms] on-site potential energy (eV) added to every orbital of
     * the atom, or NULL = 0.  It becomes the ham's per-atom potential (in
     * every storage format it is kept beside the packed blocks, not inside
     * them), so a later tbh_ham_set_potential replaces it. */
    const double* onsite_pot;
    /* host [3] Bloch vector as fractions of the box reciprocal vectors; a
     * bond that wraps by w boxes gets the phase exp(2 pi i k.w).  NULL =
     * Gamma.  A non-zero k makes H complex. */
    const double* kfrac;
    int32_t prec;             /* TBH_F64 or TBH_F32 */
    /* lanes of a wavefront that share one atom's rows (1..n_o, must divide
     * n_o); 0 = choose automatically. */
    int32_t lanes_per_atom;
    /* TBH_F32 only: also keep an FP64 copy of H for residuals and
     * Rayleigh-quotient refinement (tbh_apply_h_f64, tbh_lanczos_eigs). */
    int32_t keep_f64;
    /* TBH_F32 only: also keep the atom-major block copy the multi-vector
     * kernels read (tbh_apply_h_multi, tbh_batch_*). */
    int32_t multi_vector;
    /* 1: store each distinct bond block once, in a table indexed by
     * (sublattice, species of the atom, species of the neighbour, bond slot),
     * plus an 8-byte key record per atom, instead of four blocks per atom.
     * The Slater-Koster blocks of an unstrained real H at Gamma depend on
     * nothing else (Sec. I: two-centre nearest-neighbour form), so H.x then
     * reads about 110 instead of 1,700 bytes per atom (sp3d5s*).  Needs: no
     * bond_scale, Gamma (real H), no spin, no passivation (diagonal on-site
     * blocks), lanes_per_atom 0, no multi_vector, and a table of at most
     * 48 KB; the build verifies every atom's blocks against the table and
     * returns TBH_EINVAL otherwise.  onsite_pot becomes the ham's per-atom
     * potential (as tbh_ham_set_potential). */
    int32_t tabulated;
    /* 1: spin-diagonal bond storage for an H with spin at Gamma.  Hopping is
     * spin-independent in the two-centre form (Sec. I; the spin-orbit term of
     * the sp3d5s*+SO model sits on the atom), so every bond block is
     * I_2 (x) b with b real (n_o/2 x n_o/2, strain scale included): the
     * packed H keeps b once per bond and the full complex on-site block
     * (passivation and spin-orbit).  For sp3d5s*+SO in FP32 that is 4,800 B
     * per atom instead of 16,000.  Needs spin, Gamma (no kfrac), no
     * tabulated, lanes_per_atom 0; the build checks every bond block for the
     * I_2 (x) real form and returns TBH_EINVAL otherwise. */
    int32_t spin_diagonal;
} tbh_build_opts;

typedef struct {
    int64_t n_atoms;
    int64_t dim;              /* n_atoms * n_orb (complex elements if complex) */
    int32_t n_orb;            /* orbitals per atom, spin included */
    int32_t is_complex;
    int32_t prec;
    int32_t lanes_per_atom;
    int32_t onsite_diagonal;  /* 1 if every on-site block is diagonal */
    int32_t has_f64;          /* FP64 copy present */
    int64_t n_dangling;       /* dangling bond slots */
    int64_t stored_bytes;     /* device bytes of the packed H (main precision) */
    int64_t hx_bytes;         /* algorithmic bytes of one H.x: packed H (or
                                 key records + block table) + neighbour
                                 table + x once + y once (+ potential) */
    int32_t tabulated;        /* 1 if the bond blocks are tabulated */
    int32_t spin_diagonal;    /* 1 if the bond blocks are stored spin-diagonal */
} tbh_ham_info;

/* Pure host step of the build: neighbour table and the assembled FP64
 * blocks, written to caller-owned host arrays.  No device is touched.
 * nbr: [n][4] int32 (-1 = dangling); wrap: [n][4][3] int8;
 * onsite: [n][n_o][n_o] and bonds: [n][4][n_o][n_o] as doubles, complex
 * interleaved when H is complex (either may be NULL).  Bond block (i,b) is
 * <i,row|H|nbr(i,b),col>; the block of a B atom is exactly the conjugate
 * transpose of its partner's. */
int tbh_build_blocks_host(const tbh_geometry* g, const tbh_params* p,
                          const tbh_build_opts* o, int32_t* nbr, int8_t* wrap,
                          double* onsite, double* bonds, int32_t* is_complex);

/* Pure host step of the tabulated build (tbh_build_opts.tabulated): the
 * distinct bond blocks and per-species on-site diagonals of an unstrained
 * real H at Gamma without spin or passivation (the two-centre blocks of
 * Sec. I depend only on the species pair and the bond direction), and each
 * atom's key record, in the caller's atom order.  No device is touched.
 * table: host, table_cap doubles; on success it holds the nu blocks
 *   [nu][n_o][n_o] (block of bond (i,b) = <i,row|H|nbr(i,b),col>) followed
 *   by the on-site diagonals [n_species][n_o] without the potential; NULL
 *   writes only *n_blocks, so a caller can size the table first
 *   (nu * n_o * n_o + n_species * n_o doubles).
 * keys: host [n_atoms][8] bytes or NULL: bytes 0..3 the table index of
 *   bond slot b (255 = dangling), byte 4 the atom's species, bytes 5..7 zero.
 * n_blocks: out, nu.
 * TBH_EINVAL when the model cannot be tabulated (strain, spin, k-point,
 * passivated dangling bonds, more than 4 species) or table_cap is short. */
int tbh_tabulate_host(const tbh_geometry* g, const tbh_params* p,
                      const tbh_build_opts* o, double* table, int64_t table_cap,
                      int32_t* n_blocks, uint8_t* keys);

/* Build H on the context's device: neighbour search, Slater-Koster bond
 * blocks (strain, Bloch phase), on-site blocks (spin-orbit, passivation,
 * potential), packed into the atom-ordered block layout the kernels stream.
 * *out owns its device memory; release it with tbh_ham_destroy. */
int tbh_build_hamiltonian(tbh_ctx* ctx, const tbh_geometry* g, const tbh_params* p,
                          const tbh_build_opts* o, tbh_ham** out);
int tbh_ham_destroy(tbh_ham* h);
int tbh_ham_info_get(const tbh_ham* h, tbh_ham_info* out);
/* Host copies of the neighbour table ([n][4]) and wraps ([n][4][3]). */
int tbh_ham_neighbours(const tbh_ham* h, int32_t* nbr, int8_t* wrap);

/* Replace the per-atom on-site potential (Schrodinger-Poisson update, Sec.
 * III-A item 3): pot_dev is device [n_atoms] FP64 (eV, caller's atom order),
 * or NULL = 0.  It replaces the build-time onsite_pot as well, the same way
 * in every storage format (stored, tabulated, FP64 copy, multi-vector copy).
 * The blocks are not rebuilt; H.x adds pot[i] * x_i. */
int tbh_ham_set_potential(tbh_ham* h, const double* pot_dev);

/* y = H x.  x, y: device, [dim] scalars of the ham's precision (complex
 * interleaved).  nrhs must be 1 (see tbh_apply_h_multi).  x and y must not
 * overlap and must be 16-byte aligned. */
int tbh_apply_h(tbh_ham* h, const void* x, void* y, int32_t nrhs);

/* Y = H X for nrhs right-hand vectors on the matrix cores (FP32 inputs,
 * FP32 accumulation).  X, Y: device [n_atoms][n_orb][nrhs] FP32 (complex
 * interleaved: [..][nrhs][2]).  nrhs = 16 or 32; the ham must be TBH_F32,
 * built with multi_vector = 1. */
int tbh_apply_h_multi(tbh_ham* h, const float* X, float* Y, int32_t nrhs);
/* y = H x in FP64 with the FP64 copy (or the main copy for TBH_F64). */
int tbh_apply_h_f64(tbh_ham* h, const double* x, double* y);


/* ------------------------------------------------------------------------
 * Lanczos eigensolver (Sec. III-A, item 1; the iteration count of Sec.
 * II-B is its unit of cost).
 *
 * Recurrence (j = 0..m-1, v_0 = v0/|v0|, beta_0 = 0):
 *   w = H v_j - beta_j v_{j-1};  alpha_j = Re(v_j^H w);  w -= alpha_j v_j;
 *   [reorth: twice { c = V^H w; w -= V c } over v_0..v_j, FP64 coefficients]
 *   beta_{j+1} = |w|;  breakdown if beta_{j+1} <= 1e-12 max|T|;
 *   v_{j+1} = w / beta_{j+1}.
 * Vectors are stored in the ham's precision; every inner product,
 * reorthogonalisation coefficient and the tridiagonal eigensolve are FP64.
 * ------------------------------------------------------------------------ */
typedef struct {
    double sigma;          /* target energy (eV) */
    int32_t k;             /* distinct eigenvalues wanted (>= 1) */
    int32_t max_iter;      /* Lanczos steps m (1..100000) */
    int32_t reorth;        /* 0: none; 1: full CGS2.  tbh_lanczos_run keeps three vectors
                              without reorthogonalisation and m+1 with it; tbh_lanczos_eigs
                              always keeps all m+1 (Ritz vectors need them), i.e.
                              (m+1) * dim * element bytes of device memory. */
    int32_t n_cand;        /* Ritz pairs examined; 0 = min(m, max(4k, k+16)) */
    double res_tol;        /* converged iff |H y - theta y| <= res_tol, |y| = 1 (0 = 1e-4 eV) */
    double merge_tol;      /* converged values closer than this are one eigenvalue (0 = 1e-6 eV) */
    const double* v0;      /* host [dim] FP64 start vector (complex interleaved), not all
                              zero; or NULL to use v0_dev */
    const double* v0_dev;  /* device [dim] FP64 start vector, used when v0 is NULL */
} tbh_lanczos_opts;

typedef struct {
    int32_t steps;         /* steps taken (fewer than max_iter after a breakdown) */
    int32_t breakdown;     /* 1 if the recurrence stopped on an invariant subspace */
    int32_t n_found;       /* distinct converged eigenvalues reported (<= k) */
    int32_t n_cand;        /* Ritz pairs examined */
    double max_res;        /* largest residual among the reported values (eV) */
    double seconds;        /* wall time of the call */
    double hx_seconds;     /* device time of the H.x kernels of the recurrence (0 unless timed) */
} tbh_lanczos_report;

/* Eigenvalues nearest sigma.  Candidates are the n_cand Ritz values of T_m
 * nearest sigma; each gets its Ritz vector y = V s, an explicit FP64
 * residual |H y - theta y| and a Rayleigh-quotient refinement y^H H y with
 * the FP64 copy of H (the ham must have one: TBH_F64, or TBH_F32 built with
 * keep_f64).  Converged candidates whose refined values lie within merge_tol
 * are one eigenvalue; the k distinct converged values nearest sigma (by
 * refined value; ties: lower value) are returned in ascending order.  Without reorthogonalisation the recurrence loses
 * orthogonality once Ritz values converge and repeats them ("ghost" copies,
 * Paige's analysis); each copy converges to the same eigenvalue and is merged
 * by merge_tol, so long runs (thousands of steps, memory permitting) reach
 * interior eigenvalues at the cost of H.x alone.
 * Outputs (host, [k], may be NULL): evals = raw Ritz values, refined =
 * Rayleigh quotients, res = residuals (eV), copies = converged copies merged
 * into the value.  evecs_dev (device, may be NULL): [k][dim] FP64 unit Ritz
 * vectors (complex interleaved).  Slots past n_found are set to NaN / 0.
 * Returns TBH_ENOCONV (results written) if fewer than k values converged. */
int tbh_lanczos_eigs(tbh_ham* h, const tbh_lanczos_opts* o, double* evals, double* refined,
                     double* res, int32_t* copies, double* evecs_dev, tbh_lanczos_report* rep);

/* The recurrence only: o->max_iter steps (o->reorth) from o->v0 / o->v0_dev;
 * sigma, k and the tolerances are ignored.  alpha[m], beta[m] (host, may be
 * NULL) receive alpha_j and beta_{j+1}; entries past the last step are 0.
 * With time_hx != 0 the H.x kernels are bracketed by HIP events and their
 * summed duration is reported.  The ham keeps the Lanczos workspace between
 * calls with the same m and reorth, so repeated runs allocate nothing. */
int tbh_lanczos_run(tbh_ham* h, const tbh_lanczos_opts* o, double* alpha, double* beta,
                    int32_t time_hx, tbh_lanczos_report* rep);

/* ------------------------------------------------------------------------
 * Block Lanczos (Sec. III-A, item 1 names "(block) Lanczos").
 *
 * A block of b orthonormal vectors replaces the single vector, so an
 * eigenvalue of multiplicity up to b (degenerate states of a symmetric
 * structure) appears with its full multiplicity, and a start block can carry
 * several approximate eigenvectors (warm starts).  With Q_1 B_0 = X0:
 *   W = H Q_j - Q_{j-1} B_j^T;  A_j = Q_j^T W;  W -= Q_j A_j;
 *   twice { W -= Q (Q^T W) } over Q_1..Q_j;  Q_{j+1} B_{j+1} = W (QR);
 * Rayleigh-Ritz on the block-tridiagonal T_m; Ritz vectors Y = Q S with
 * explicit FP64 residuals |H y - theta y| and Rayleigh quotients (FP64 copy
 * of H).  H.X and the basis are FP32 on the matrix cores; inner products,
 * coefficients, QR factors, T and its eigensolve are FP64.  A QR column whose
 * remainder is at most defl_tol |H| is deflated and replaced by a SplitMix64
 * vector (counter ((j b + i) << 32) + row) orthogonalised against the basis.
 * Real H only (TBH_F32 built with multi_vector = 1 and keep_f64 = 1).
 * ------------------------------------------------------------------------ */
typedef struct {
    double sigma;          /* target energy (eV) */
    int32_t block;         /* block size b: 16, 32 or 64 */
    int32_t steps;         /* block steps m per run; m * b <= 2048 */
    int32_t cycles;        /* runs at most; a later run restarts from the b Ritz vectors nearest sigma */
    int32_t k;             /* Ritz pairs wanted, 1 <= k <= b; each copy of a repeated eigenvalue counts */
    double res_tol;        /* converged iff |H y - theta y| <= res_tol, |y| = 1 (0 = 1e-4 eV) */
    double defl_tol;       /* deflation threshold relative to |H| (0 = 1e-6) */
    const double* x0_dev;  /* device [b][dim] FP64 start block (state-major), or NULL for a
                              SplitMix64 block */
    int32_t fold;          /* 0: Krylov space of H.  1: of (H - sigma)^2 (two H.X per block step):
                              the pairs nearest sigma are then its smallest eigenvalues, so
                              interior pairs next to a gap converge without spurious Ritz values
                              in the gap; eigenvalues are the FP64 Rayleigh quotients of H */
} tbh_block_lanczos_opts;

typedef struct {
    int32_t cycles;        /* runs made */
    int32_t n_found;       /* converged pairs reported (<= k) */
    int32_t deflated;      /* deflated QR columns over all runs */
    double max_res;        /* largest residual among the reported pairs (eV) */
    double seconds;        /* wall time of the call */
    double hx_seconds;     /* device time of the multi-vector H.X launches */
} tbh_block_lanczos_report;

/* The k Ritz pairs nearest sigma.  Each run computes the b Ritz pairs
 * nearest sigma; the call stops when the k of them nearest sigma (by Ritz
 * value) have converged, or after o->cycles runs.  The k converged pairs
 * nearest sigma are returned ascending by Rayleigh quotient (host [k]:
 * evals = Ritz values, refined = Rayleigh quotients, res = residuals;
 * evecs_dev: device [k][dim] FP64 unit vectors, or NULL); slots past
 * n_found are NaN / 0, and the call returns TBH_ENOCONV.  Device memory:
 * (m + 3) * dim * b * 4 bytes for the basis and work blocks plus b * dim * 8
 * for the Ritz vectors. */
int tbh_block_lanczos_eigs(tbh_ham* h, const tbh_block_lanczos_opts* o, double* evals, double* refined,
                           double* res, double* evecs_dev, tbh_block_lanczos_report* rep);

/* ------------------------------------------------------------------------
 * Filtered subspace eigensolver for the states next to a gap (the
 * self-consistent loop's eigen-solve, Sec. III-A items 1-3).
 *
 * With F = (H - sigma)^2 and sigma in the gap, the pairs nearest sigma are
 * the smallest eigenvalues of F.  A block of b vectors is filtered by the
 * scaled Chebyshev polynomial of F that damps [f_cut, f_max] (f_cut the
 * largest F value the block represents, f_max from spectral bounds of H by
 * 60 Lanczos steps), orthonormalised by Cholesky QR and rotated to the Ritz
 * vectors of H on its span (Chebyshev-filtered subspace iteration: Zhou,
 * Saad, Tiago, Chelikowsky, J. Comput. Phys. 219 (2006) 172).  Each degree
 * costs two multi-vector H.X (FP32 on the matrix cores); Gram and
 * Rayleigh-Ritz matrices and residual sums are FP64.  Real H built TBH_F32
 * with multi_vector = 1.  x0_dev = NULL starts from a random block; pass the
 * vectors of an earlier call (padded to b) to warm-start.
 * ------------------------------------------------------------------------ */
typedef struct {
    double sigma;          /* fold centre (eV): in the gap, nearer the wanted pairs than any other band */
    int32_t block;         /* b: 16, 32 or 64 */
    int32_t degree;        /* Chebyshev degree of each filter after the first (>= 1) */
    int32_t degree_cold;   /* degree of the first filter from a random block */
    int32_t max_iter;      /* filter iterations at most */
    int32_t k;             /* pairs nearest sigma that must converge, 1 <= k <= b */
    double res_tol;        /* |H y - theta y| / |y| <= res_tol (0 = 1e-4 eV) */
    const double* x0_dev;  /* device [b][dim] FP64 start block (state-major), or NULL for a
                              SplitMix64 block */
} tbh_filter_opts;

typedef struct {
    int32_t iterations;    /* filter iterations made */
    int32_t n_found;       /* converged pairs reported (<= k) */
    double max_res;        /* largest residual among them (eV) */
    double emin, emax;     /* spectral bounds used (eV) */
    double seconds;
} tbh_filter_report;

/* The k converged pairs nearest sigma, ascending: evals (host [k]), res
 * (host [k]), evecs_dev (device [k][dim] FP64 unit vectors, or NULL); slots
 * past n_found are NaN / 0 and the call returns TBH_ENOCONV. */
int tbh_filtered_eigs(tbh_ham* h, const tbh_filter_opts* o, double* evals, double* res, double* evecs_dev,
                      tbh_filter_report* rep);

/* The nc eigenpairs nearest sigma of the real symmetric n x n matrix A (host,
 * row-major, n <= 2048) by the projected-matrix eigensolver of block Lanczos
 * (FP64 Householder tridiagonalisation, bisection, inverse iteration,
 * back-transformation on the context's device): theta (host [nc],
 * ascending) and vecs (host [nc][n] orthonormal eigenvectors, or NULL). */
int tbh_symm_eig_near(tbh_ctx* ctx, int32_t n, const double* A, double sigma, int32_t nc, double* theta,
                      double* vecs);

/* Eigenvalues (ascending) of the symmetric tridiagonal matrix with diagonal
 * diag[m] and off-diagonal off[m-1] (host arrays), by FP64 Sturm bisection
 * on the context's device; theta[m] is host output. */
int tbh_tridiag_eig(tbh_ctx* ctx, int32_t m, const double* diag, const double* off, double* theta);

/* ------------------------------------------------------------------------
 * Finite-difference Poisson solver (Sec. III-A, item 3).
 *
 * Grid nodes [nz][ny][nx] with spacing h_nm, periodic in x and y, phi = 0 on
 * the ghost planes z = -1 and z = nz; 7-point Laplacian:
 *   -eps0 eps_r Lap_h phi = rho    (phi in V, rho in e/nm^3)
 * ------------------------------------------------------------------------ */

/* FP64 conjugate gradients for phi.  rho_dev, phi_dev: device
 * [nz][ny][nx] FP64; phi_dev holds the initial guess on entry and the
 * solution on return.  Stops when |r| <= rel_tol |b| or after max_iter
 * iterations (then TBH_ENOCONV with the partial solution written). */
int tbh_poisson_solve(tbh_ctx* ctx, const int32_t grid[3], double h_nm, double eps_r, const double* rho_dev,
                      double* phi_dev, double rel_tol, int32_t max_iter, int32_t* iters,
                      double* rel_res);

/* The same solve without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, result and status as tbh_poisson_solve;
 * additionally TBH_EINVAL when nx*ny*nz exceeds 262,144 (2^18) nodes.  Its
 * scratch (b, the CG vectors r, p, Ap and reduction partials: 8.5 MB) is one
 * static device array per GPU, held until the process ends and shared by
 * every call on that GPU: calls that overlap on one GPU (several streams or
 * threads) race on it. */
int tbh_poisson_solve_noalloc(tbh_ctx* ctx, const int32_t grid[3], double h_nm, double eps_r,
                              const double* rho_dev, double* phi_dev, double rel_tol, int32_t max_iter,
                              int32_t* iters, double* rel_res);

/* ------------------------------------------------------------------------
 * Self-consistent Schrodinger-Poisson loop (Sec. III-A; the application of
 * Sec. III-B is a P delta layer in Si at 4 K).
 *
 * One step with input potential energy U (eV, on the grid; atom (qx,qy,qz)
 * sits on node (qx,qy,qz)):
 *  1. H(U) = H_TB + U at every atom's orbitals;
 *  2. Lanczos (full CGS2, lanczos_iter steps) targeted 0.05 eV below the
 *     lowest filled state of the previous step (first step, or none filled:
 *     e_cbm + the 1st percentile of U over the atoms); the n_cand Ritz pairs
 *     nearest the target with residual
 *     <= res_tol are the states, their energies the FP64 Rayleigh quotients;
 *  3. conduction-band-like states (E - <psi|U|psi> > sigma_mid) are filled
 *     with spin degeneracy 2 and Fermi-Dirac occupation at T_K; the Fermi
 *     level comes from neutrality (2 sum f = n_donors) unless fermi_fixed is
 *     given (not NaN);
 *  4. rho = e (donors - electrons) / h^3 at the nodes, U_out = -phi from the
 *     Poisson solve (CG from the previous solution);
 *  5. residual = max |U_out - U|; U <- U + mix_alpha (U_out - U).
 * ------------------------------------------------------------------------ */
typedef struct tbh_scf tbh_scf;

typedef struct {
    int32_t grid[3];          /* nx, ny, nz nodes (must contain every atom position) */
    double h_nm;              /* grid spacing in nm (a/4 for the Si lattice) */
    double eps_r;             /* relative permittivity */
    double T_K;               /* temperature; 0 = step occupation */
    double mix_alpha;         /* linear mixing factor, (0, 1] */
    double tol_eV;            /* converged when max |U_out - U| < tol_eV */
    double sigma_mid;         /* gap centre of the bulk bands (CB-like test) */
    double e_cbm;             /* bulk conduction-band minimum (Lanczos target offset) */
    double fermi_fixed;       /* NaN: Fermi level from neutrality; else this Fermi level */
    int32_t n_cand;           /* Ritz pairs per eigen-solve */
    int32_t lanczos_iter;     /* Lanczos steps per eigen-solve (>= n_cand, <= 4000) */
    double res_tol;           /* residual (eV) for a Ritz pair to count as a state */
    double cg_tol;            /* Poisson CG relative residual */
    int32_t cg_max_iter;
    const int32_t* donor_atoms;  /* host [n_donors]: atoms carrying a +e donor ion */
    int32_t n_donors;         /* also the electron count (neutrality) */
    const double* v0;         /* host [dim] FP64 Lanczos start vector (complex interleaved) */
    /* eigen-solve: 0 = Lanczos with full CGS2 (n_cand, lanczos_iter, res_tol as
     * above); 1 = filtered subspace iteration (tbh_filtered_eigs) on a block of
     * `block` vectors kept across steps (real H built with multi_vector = 1):
     * the fold centre is three quarters of the way from the valence-band top
     * estimate (e_vbm + max U) to the conduction-band bottom estimate (the
     * previous step's lowest filled state, or e_cbm + the 1st percentile of U
     * over the atoms); each step runs
     * filters of degree filter_degree (filter_degree_cold on the first step,
     * from a random block) until the k_states pairs nearest the centre have
     * residual <= max(res_tol, 0.1 * the previous step's SCF residual) (0.01 *
     * with update_mode 1; max(res_tol, 0.01 eV) on the first step), at least
     * one and at most filter_max_iter per step (see filter_max_iter_cold for the
     * first); on a warm step with linear mixing the first filter's damping
     * bound comes from the Ritz values the previous step ended with; every
     * state of the block takes part in the filling. */
    int32_t eig_mode;
    int32_t block;            /* 16, 32 or 64 */
    int32_t filter_degree;
    int32_t filter_degree_cold;
    int32_t filter_max_iter;
    int32_t k_states;         /* <= block */
    double e_vbm;             /* bulk valence-band maximum (eV) */
    /* update of step 5: 0 = linear mixing; 1 = Newton-Raphson on
     * G(U) = A U - kappa (n(U) - N_D) = 0 (A = -Lap_h, kappa = 1 / (h^3 eps0
     * eps_r); Sec. III-A obtains the potential by Newton-Raphson).  The
     * Jacobian J = A - kappa chi takes the density response chi = dn/dU of
     * first-order perturbation theory over the newton_states lowest filled-
     * class (CB-like) states of the step,
     *   chi v = 2 sum_ik g_ik rho_ik (rho_ik . v) - 2 d (d . v) / sum_i f'_i,
     *   rho_ik(atom) = sum_alpha psi_i psi_k, g_ik = (f_i - f_k)/(E_i - E_k),
     *   g_ii = f'_i, d = sum_i f'_i rho_ii (the last term only under
     *   neutrality),
     * with occupations smeared at newton_kT (eV) inside chi only; J d = -G is
     * solved by Jacobi-preconditioned CG (FP64) to newton_cg_tol, and the
     * steps are combined by Anderson mixing over the last anderson_depth
     * steps.  The residual and the stopping rule stay those of step 5.
     * Real H only. */
    int32_t update_mode;
    int32_t newton_states;    /* 1..128 */
    double newton_kT;         /* > 0 */
    int32_t anderson_depth;   /* 0..8 */
    double newton_cg_tol;
    int32_t newton_cg_max_iter;
    /* eig_mode 1 with linear mixing: at most this many filter passes in the
     * loop's first (cold) eigen-solve, from the random block, when the start is
     * the zero potential; 0 = filter_max_iter.  From the zero start the next
     * steps' tolerance follows a large first residual, so that solve's
     * accuracy is mostly unused; a built start (mean, learned, any potential
     * set) and the Newton-Raphson update keep the full filter_max_iter
     * (measured on the 8x8x60-cell slab). */
    int32_t filter_max_iter_cold;
} tbh_scf_opts;

typedef struct {
    int32_t iterations;       /* steps taken so far */
    int32_t converged;        /* residual < tol_eV at the last step */
    double residual;          /* max |U_out - U| of the last step (eV) */
    double fermi;             /* Fermi level (eV) */
    int32_t n_cb;             /* states filled (CB-like, converged) */
    int32_t n_conv;           /* converged Ritz pairs */
    double electrons;         /* 2 sum f over the filled states */
    int32_t cg_iters;
    double cg_rel_res;
    int32_t lanczos_steps;
    double u_min;             /* min U after the update (eV) */
    double sigma;             /* Lanczos target of the step (eV) */
    double seconds, eig_seconds, poisson_seconds;
    int32_t fell_back;        /* 1 if this step abandoned a start potential for the zero start */
    int32_t newton_cg_iters;  /* update_mode 1: CG iterations of the Newton solve (0 otherwise) */
    int32_t newton_pairs;     /* update_mode 1: state pairs in chi after pruning */
    double newton_seconds;    /* update_mode 1: time of the update */
} tbh_scf_report;

/* The SCF object keeps h (which must outlive it, and must have an FP64 copy)
 * and owns its grid buffers.  The start potential is zero. */
int tbh_scf_create(tbh_ham* h, const tbh_scf_opts* o, tbh_scf** out);
int tbh_scf_destroy(tbh_scf* s);
/* Set U (device [nz][ny][nx] FP64, eV), or NULL = 0 (the plain start). */
int tbh_scf_set_potential(tbh_scf* s, const double* U_dev);
/* Start potential of the loop (Sec. III-A starts it from a given potential).
 *  kind 0: zero.
 *  kind 1 (mean): U0 = U_bare + mean.
 *  kind 2 (learned): U0 = U_bare + mean + scale * y, y = net(x) or, with
 *    symmetrize, the average of op^-1 net(op x) over the four in-plane point
 *    operations of the slab that map each sublattice onto itself (identity,
 *    the (110) and (1-10) mirrors, the two-fold rotation about the atom at
 *    the origin; needs nx = ny).  The input x (4 channels) is built on the
 *    device: the donor count per node, the A- and B-sublattice occupation of
 *    the nodes, and U_bare / feat_scale.
 * U_bare is the electron potential energy of the donor charges alone (the
 * loop's Poisson solve of its donor term, CG to 1e-12); mean (device FP32
 * [nz][ny][nx]) and scale are the training mean and scale of U* - U_bare.
 * The start is abandoned for the zero start (reported as fell_back by the
 * step that does it) when a residual is not finite, the residual grows three
 * steps in a row, or the first residual exceeds first_res_limit (0 = no
 * limit). */
typedef struct tbh_net tbh_net;
typedef struct {
    int32_t kind;             /* 0 zero, 1 mean, 2 learned */
    tbh_net* net;             /* kind 2: 4 input channels, the loop's grid */
    const float* mean_dev;    /* kinds 1, 2 */
    double scale;             /* kind 2 */
    double feat_scale;        /* kind 2 */
    int32_t symmetrize;       /* kind 2 */
    double first_res_limit;
} tbh_scf_start;
int tbh_scf_set_start(tbh_scf* s, const tbh_scf_start* start);
/* Copy the current U into U_dev (device [nz][ny][nx] FP64). */
int tbh_scf_get_potential(tbh_scf* s, double* U_dev);
/* Electrons per atom of the last step's filling (device [n_atoms] FP64,
 * caller's atom order): sum over the filled states of 2 f sum_alpha
 * |psi(i, alpha)|^2. */
int tbh_scf_get_density(tbh_scf* s, double* n_dev);
/* One self-consistency step; rep (host) receives the step's report. */
int tbh_scf_step(tbh_scf* s, tbh_scf_report* rep);
/* Steps until converged or max_iter steps; TBH_ENOCONV if not converged. */
int tbh_scf_run(tbh_scf* s, int32_t max_iter, tbh_scf_report* rep);

/* ------------------------------------------------------------------------
 * Batched multi-vector H.X: many Hamiltonians of uneven size (cells x
 * k-points; the k-space groups of Sec. II-C) in one persistent launch,
 * captured in a HIP graph.
 * ------------------------------------------------------------------------ */
typedef struct tbh_batch tbh_batch;

/* hams[count] (same orbital count and complex-ness, TBH_F32, multi_vector),
 * X[count], Y[count]: device buffers as in tbh_apply_h_multi.  The batch
 * keeps the pointers (which must stay valid) and a captured graph of the
 * launch.  grid / remap: persistent workgroups and their walk over the
 * concatenated atoms (defaults: 8 workgroups per CU, remap 1): remap 0 = one
 * grid-wide window of consecutive atoms in workgroup order; 1 = the same
 * window with each XCD holding a contiguous part of it; 2 = each XCD owns a
 * contiguous eighth of the atoms, swept by its own workgroups. */
int tbh_batch_create(tbh_ctx* ctx, tbh_ham* const* hams, int32_t count, const float* const* X, float* const* Y,
                     int32_t nrhs, tbh_batch** out);
int tbh_batch_destroy(tbh_batch* b);
/* Launch the captured graph on the context's stream (asynchronous). */
int tbh_batch_apply(tbh_batch* b);
/* The same work as one kernel launch per Hamiltonian (the reference point). */
int tbh_batch_apply_separate(tbh_batch* b);
/* Choose the launch configuration by timing candidates on the device (or
 * read it from cache_path when it holds an entry for this batch shape);
 * the chosen configuration is written back to cache_path (may be NULL) and
 * the graph is re-captured.  best_ms (may be NULL) receives the time of one
 * batched application with the chosen configuration. */
int tbh_batch_autotune(tbh_batch* b, const char* cache_path, int32_t* grid, int32_t* remap, double* best_ms);
/* Set the launch configuration explicitly (re-captures the graph). */
int tbh_batch_configure(tbh_batch* b, int32_t grid, int32_t remap);

/* ------------------------------------------------------------------------
 * Learned start potential for the self-consistent loop (Sec. III-A starts
 * it from a given potential): a 3-D convolutional network maps input maps
 * of the donor layout to the potential.
 *
 * n_layers 3x3x3 convolutions c_in -> 32 -> ... -> 32 -> 1 (c_in = 1 or 4,
 * 2 <= n_layers <= 8) with one dilation per layer, ReLU after all but the
 * last, circular padding along x and y, zero padding along z; FP16
 * activations and weights on the matrix cores with FP32 accumulation, FP32
 * master weights and Adam (beta 0.9 / 0.999, eps 1e-8).
 * Parameters (host, FP32) in canonical order: for each layer, W[c_out][c_in]
 * [dz][dy][dx] then b[c_out].  Inputs are device FP32 [c_in][nz][ny][nx],
 * outputs device FP32 [nz][ny][nx].
 * ------------------------------------------------------------------------ */
/* channels must be 32; dilations: host [n_layers] in 1..64, or NULL for the
 * default 4-layer (1, 2, 4, 1); grid = (nx, ny, nz). */
int tbh_net_create(tbh_ctx* ctx, int32_t channels, int32_t in_channels, int32_t n_layers,
                   const int32_t* dilations, const int32_t grid[3], tbh_net** out);
int tbh_net_destroy(tbh_net* n);
int tbh_net_num_params(const tbh_net* n, int64_t* count);
/* Copy parameters in (resets the Adam moments) or out (host FP32). */
int tbh_net_set_params(tbh_net* n, const float* params);
int tbh_net_get_params(tbh_net* n, float* params);
/* y = net(x). */
int tbh_net_forward(tbh_net* n, const float* x_dev, float* y_dev);
/* Per-voxel weights w of the training loss mean(w (net(x) - t)^2): device
 * FP32 [nz][ny][nx], copied into the net; NULL restores w = 1. */
int tbh_net_set_loss_weights(tbh_net* n, const float* w_dev);
/* Gradient of the loss mean(w (net(x) - t)^2) w.r.t. the parameters (host,
 * canonical order) and the loss. */
int tbh_net_gradients(tbh_net* n, const float* x_dev, const float* t_dev, float* grad, double* loss);
/* One Adam step on the mean loss over a batch of (x[i], t[i]) device maps;
 * loss = mean over the batch before the step.  When the loss or any
 * gradient entry is not finite (an overflow of the half-precision
 * activations or their gradients) the step is skipped: weights, moments and
 * the step count stay as they were, and loss reports the non-finite value
 * or the loss of the skipped batch. */
int tbh_net_train_step(tbh_net* n, const float* const* x_dev, const float* const* t_dev, int32_t batch,
                       double lr, double* loss);

#ifdef __cplusplus
}
#endif

#endif /* TBH_H */
