// Host model builder: input validation, neighbour table, Slater-Koster bond
// blocks in closed form, on-site blocks, and packing into the layout the
// H.x kernels stream.
//
// The model is the empirical sp3s* / sp3d5s* nearest-neighbour tight-binding
// Hamiltonian with strain named in the paper's Abstract and Sec. I.  The
// two-centre bond blocks follow the closed-form table of Slater & Koster
// (Phys. Rev. 94, 1498 (1954), Table I) in the direction cosines (l, m, n)
// of the bond.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <exception>
#include <thread>

#include "tbh_internal.h"

namespace tbh {

namespace {

constexpr int kSlot[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

enum { SS, SSTSST, SSST, SP, SSTP, SD, SSTD, PPS, PPP, PDS, PDP, DDS, DDP, DDD };

}  // namespace

void sk_block_closed_form(int model, const double* V, double l, double m, double n, double* E) {
    const int nb = model == TBH_SP3S ? 5 : 10;
    const int s = 0, st = nb - 1;
    const int p0 = 1;
    std::memset(E, 0, sizeof(double) * nb * nb);
    auto at = [&](int a, int b) -> double& { return E[a * nb + b]; };
    const double dc[3] = {l, m, n};
    at(s, s) = V[SS];
    at(st, st) = V[SSTSST];
    at(s, st) = at(st, s) = V[SSST];
    for (int a = 0; a < 3; ++a) {
        at(s, p0 + a) = dc[a] * V[SP];
        at(p0 + a, s) = -dc[a] * V[SP];
        at(st, p0 + a) = dc[a] * V[SSTP];
        at(p0 + a, st) = -dc[a] * V[SSTP];
        for (int b = 0; b < 3; ++b)
            at(p0 + a, p0 + b) = dc[a] * dc[b] * (V[PPS] - V[PPP]) + (a == b ? V[PPP] : 0.0);
    }
    if (model == TBH_SP3S) return;

    const double r3 = std::sqrt(3.0);
    const double l2 = l * l, m2 = m * m, n2 = n * n;
    const double lmn = l * m * n;
    const double lm2 = l2 - m2;           // l^2 - m^2
    const double z2 = n2 - 0.5 * (l2 + m2);
    enum { XY = 4, YZ = 5, ZX = 6, X2 = 7, Z2 = 8 };
    // s-d and s*-d (even parity: symmetric)
    const double fsd[5] = {r3 * l * m, r3 * m * n, r3 * n * l, 0.5 * r3 * lm2, z2};
    for (int d = 0; d < 5; ++d) {
        at(s, XY + d) = at(XY + d, s) = fsd[d] * V[SD];
        at(st, XY + d) = at(XY + d, st) = fsd[d] * V[SSTD];
    }
    // p-d (odd parity: E_dp = -E_pd)
    const double ps = V[PDS], pp = V[PDP];
    double pd[3][5];
    pd[0][0] = r3 * l2 * m * ps + m * (1 - 2 * l2) * pp;        // x, xy
    pd[1][0] = r3 * m2 * l * ps + l * (1 - 2 * m2) * pp;        // y, xy
    pd[2][0] = r3 * lmn * ps - 2 * lmn * pp;                    // z, xy
    pd[0][1] = r3 * lmn * ps - 2 * lmn * pp;                    // x, yz
    pd[1][1] = r3 * m2 * n * ps + n * (1 - 2 * m2) * pp;        // y, yz
    pd[2][1] = r3 * n2 * m * ps + m * (1 - 2 * n2) * pp;        // z, yz
    pd[0][2] = r3 * l2 * n * ps + n * (1 - 2 * l2) * pp;        // x, zx
    pd[1][2] = r3 * lmn * ps - 2 * lmn * pp;                    // y, zx
    pd[2][2] = r3 * n2 * l * ps + l * (1 - 2 * n2) * pp;        // z, zx
    pd[0][3] = 0.5 * r3 * l * lm2 * ps + l * (1 - lm2) * pp;    // x, x2-y2
    pd[1][3] = 0.5 * r3 * m * lm2 * ps - m * (1 + lm2) * pp;    // y, x2-y2
    pd[2][3] = 0.5 * r3 * n * lm2 * ps - n * lm2 * pp;          // z, x2-y2
    pd[0][4] = l * z2 * ps - r3 * l * n2 * pp;                  // x, 3z2-r2
    pd[1][4] = m * z2 * ps - r3 * m * n2 * pp;                  // y, 3z2-r2
    pd[2][4] = n * z2 * ps + r3 * n * (l2 + m2) * pp;           // z, 3z2-r2
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 5; ++d) {
            at(p0 + a, XY + d) = pd[a][d];
            at(XY + d, p0 + a) = -pd[a][d];
        }
    // d-d (symmetric)
    const double ds = V[DDS], dp = V[DDP], dd = V[DDD];
    double q[5][5];
    q[0][0] = 3 * l2 * m2 * ds + (l2 + m2 - 4 * l2 * m2) * dp + (n2 + l2 * m2) * dd;
    q[1][1] = 3 * m2 * n2 * ds + (m2 + n2 - 4 * m2 * n2) * dp + (l2 + m2 * n2) * dd;
    q[2][2] = 3 * n2 * l2 * ds + (n2 + l2 - 4 * n2 * l2) * dp + (m2 + n2 * l2) * dd;
    q[0][1] = 3 * l * m2 * n * ds + l * n * (1 - 4 * m2) * dp + l * n * (m2 - 1) * dd;
    q[1][2] = 3 * m * n2 * l * ds + m * l * (1 - 4 * n2) * dp + m * l * (n2 - 1) * dd;
    q[0][2] = 3 * l2 * m * n * ds + m * n * (1 - 4 * l2) * dp + m * n * (l2 - 1) * dd;
    q[0][3] = 1.5 * l * m * lm2 * ds - 2 * l * m * lm2 * dp + 0.5 * l * m * lm2 * dd;
    q[1][3] = 1.5 * m * n * lm2 * ds - m * n * (1 + 2 * lm2) * dp + m * n * (1 + 0.5 * lm2) * dd;
    q[2][3] = 1.5 * n * l * lm2 * ds + n * l * (1 - 2 * lm2) * dp - n * l * (1 - 0.5 * lm2) * dd;
    q[0][4] = r3 * l * m * z2 * ds - 2 * r3 * l * m * n2 * dp + 0.5 * r3 * l * m * (1 + n2) * dd;
    q[1][4] = r3 * m * n * z2 * ds + r3 * m * n * (l2 + m2 - n2) * dp - 0.5 * r3 * m * n * (l2 + m2) * dd;
    q[2][4] = r3 * l * n * z2 * ds + r3 * l * n * (l2 + m2 - n2) * dp - 0.5 * r3 * l * n * (l2 + m2) * dd;
    q[3][3] = 0.75 * lm2 * lm2 * ds + (l2 + m2 - lm2 * lm2) * dp + (n2 + 0.25 * lm2 * lm2) * dd;
    q[3][4] = 0.5 * r3 * lm2 * z2 * ds - r3 * n2 * lm2 * dp + 0.25 * r3 * (1 + n2) * lm2 * dd;
    q[4][4] = z2 * z2 * ds + 3 * n2 * (l2 + m2) * dp + 0.75 * (l2 + m2) * (l2 + m2) * dd;
    for (int a = 0; a < 5; ++a)
        for (int b = a; b < 5; ++b) at(XY + a, XY + b) = at(XY + b, XY + a) = q[a][b];
}

void host_prepare(const tbh_geometry* g, const tbh_params* p, const tbh_build_opts* o,
                  HostModel& M) {
    TBH_REQUIRE(g && p && o, "null geometry, parameters or options");
    TBH_REQUIRE(g->n_atoms > 0, "n_atoms must be positive");
    TBH_REQUIRE(g->pos_q && g->species, "null positions or species");
    TBH_REQUIRE(p->model == TBH_SP3S || p->model == TBH_SP3D5S, "model must be TBH_SP3S or TBH_SP3D5S");
    TBH_REQUIRE(p->spin == 0 || p->spin == 1, "spin must be 0 or 1");
    TBH_REQUIRE(p->n_species >= 1 && p->n_species <= 16, "n_species must be in 1..16");
    TBH_REQUIRE(p->onsite && p->sk, "null on-site or two-centre parameters");
    TBH_REQUIRE(o->prec == TBH_F64 || o->prec == TBH_F32, "prec must be TBH_F64 or TBH_F32");
    const int ns = p->n_species;
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int k = 0; k < 14; ++k)
                TBH_REQUIRE(p->sk[(a * ns + b) * 14 + k] == p->sk[(b * ns + a) * 14 + k],
                            "two-centre parameters must be symmetric in the species pair");
    int64_t box[3];
    for (int ax = 0; ax < 3; ++ax) {
        box[ax] = g->box_q[ax];
        TBH_REQUIRE(box[ax] > 0, "box edges must be positive");
        TBH_REQUIRE(g->periodic[ax] == 0 || g->periodic[ax] == 1, "periodic flags must be 0 or 1");
        TBH_REQUIRE(!g->periodic[ax] || box[ax] % 4 == 0,
                    "a periodic box edge must be a whole number of cells (multiple of 4)");
    }
    TBH_REQUIRE(box[0] * box[1] * box[2] < (int64_t(1) << 32), "box too large for the index grid");

    const int64_t N = g->n_atoms;
    M.n = N;
    M.n_base = p->model == TBH_SP3S ? 5 : 10;
    M.spin = p->spin != 0;
    M.n_o = M.n_base * (M.spin ? 2 : 1);
    M.par = *p;
    M.onsite_par.assign(p->onsite, p->onsite + ns * 4);
    M.sk_par.assign(p->sk, p->sk + ns * ns * 14);
    M.so_par.assign(ns, 0.0);
    if (p->so_delta)
        for (int s = 0; s < ns; ++s) M.so_par[s] = p->so_delta[s];
    M.species.assign(g->species, g->species + N);
    for (int64_t i = 0; i < N; ++i)
        TBH_REQUIRE(M.species[i] < ns, "species index out of range at atom " + std::to_string(i));
    M.bond_scale.clear();
    if (o->bond_scale) M.bond_scale.assign(o->bond_scale, o->bond_scale + N * 4);
    M.pot.clear();
    if (o->onsite_pot) M.pot.assign(o->onsite_pot, o->onsite_pot + N);
    bool kz = true;
    for (int ax = 0; ax < 3; ++ax) {
        M.kfrac[ax] = o->kfrac ? o->kfrac[ax] : 0.0;
        if (M.kfrac[ax] != 0.0) kz = false;
    }
    M.cplx_h = M.spin || !kz;

    // sublattice and position checks; index grid position -> atom
    M.sub.assign(N, 0);
    std::vector<int32_t> grid(size_t(box[0] * box[1] * box[2]), -1);
    TBH_REQUIRE(N < (int64_t(1) << 31), "too many atoms");
    for (int64_t i = 0; i < N; ++i) {
        const int32_t* q = g->pos_q + 3 * i;
        for (int ax = 0; ax < 3; ++ax)
            TBH_REQUIRE(q[ax] >= 0 && q[ax] < box[ax],
                        "atom " + std::to_string(i) + " lies outside the box");
        const bool even = (q[0] % 2 == 0) && (q[1] % 2 == 0) && (q[2] % 2 == 0);
        const bool odd = (q[0] % 2 == 1) && (q[1] % 2 == 1) && (q[2] % 2 == 1);
        const int r = (q[0] + q[1] + q[2]) % 4;
        if (even && r == 0)
            M.sub[i] = 0;
        else if (odd && r == 3)
            M.sub[i] = 1;
        else
            throw Error(TBH_EINVAL, "atom " + std::to_string(i) + " is not on the diamond lattice");
        int32_t& cell = grid[size_t((q[2] * box[1] + q[1]) * box[0] + q[0])];
        TBH_REQUIRE(cell < 0, "duplicate atom position at atom " + std::to_string(i));
        cell = int32_t(i);
    }
    M.nbr.assign(N * 4, -1);
    M.wrap.assign(N * 12, 0);
    M.n_dangling = 0;
    for (int64_t i = 0; i < N; ++i) {
        const int32_t* q = g->pos_q + 3 * i;
        const int sg = M.sub[i] == 0 ? 1 : -1;
        for (int b = 0; b < 4; ++b) {
            int64_t t[3];
            int w[3] = {0, 0, 0};
            bool inside = true;
            for (int ax = 0; ax < 3; ++ax) {
                t[ax] = q[ax] + sg * kSlot[b][ax];
                if (t[ax] < 0 || t[ax] >= box[ax]) {
                    if (g->periodic[ax]) {
                        w[ax] = t[ax] < 0 ? -1 : 1;
                        t[ax] -= w[ax] * box[ax];
                    } else {
                        inside = false;
                    }
                }
            }
            int32_t j = -1;
            if (inside) j = grid[size_t((t[2] * box[1] + t[1]) * box[0] + t[0])];
            M.nbr[i * 4 + b] = j;
            if (j < 0) {
                ++M.n_dangling;
                continue;
            }
            for (int ax = 0; ax < 3; ++ax) M.wrap[(i * 4 + b) * 3 + ax] = int8_t(w[ax]);
        }
    }
}

namespace {

// Bond block of an A atom i in slot b (n_o x n_o), strain and phase applied.
void a_bond_block(const HostModel& M, int64_t i, int b, cplx* out) {
    const int nb = M.n_base, no = M.n_o;
    const int64_t j = M.nbr[i * 4 + b];
    const int ns = M.par.n_species;
    const double* V = &M.sk_par[(size_t(M.species[i]) * ns + M.species[j]) * 14];
    const double inv = 1.0 / std::sqrt(3.0);
    double E[100];
    sk_block_closed_form(M.par.model, V, kSlot[b][0] * inv, kSlot[b][1] * inv, kSlot[b][2] * inv, E);
    double f = M.bond_scale.empty() ? 1.0 : M.bond_scale[i * 4 + b];
    cplx ph(1.0, 0.0);
    if (M.cplx_h) {
        const int8_t* w = &M.wrap[(i * 4 + b) * 3];
        const double arg = 2.0 * M_PI * (M.kfrac[0] * w[0] + M.kfrac[1] * w[1] + M.kfrac[2] * w[2]);
        ph = cplx(std::cos(arg), std::sin(arg));
    }
    for (int k = 0; k < no * no; ++k) out[k] = 0.0;
    for (int sp = 0; sp < (M.spin ? 2 : 1); ++sp)
        for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c)
                out[(sp * nb + r) * no + sp * nb + c] = (f * E[r * nb + c]) * ph;
}

}  // namespace

void host_atom_blocks(const HostModel& M, int64_t i, cplx* D, cplx* B) {
    const int nb = M.n_base, no = M.n_o;
    const int sp_i = M.species[i];
    const double* E = &M.onsite_par[size_t(sp_i) * 4];
    // on-site: orbital energies + potential
    double e0[10];
    e0[0] = E[0];
    for (int a = 1; a < 4; ++a) e0[a] = E[1];
    if (nb == 10)
        for (int a = 4; a < 9; ++a) e0[a] = E[2];
    e0[nb - 1] = E[3];
    const double U = M.pot.empty() ? 0.0 : M.pot[i];
    double D0[100] = {0};
    for (int a = 0; a < nb; ++a) D0[a * nb + a] = e0[a] + U;
    // dangling-bond sp3 hybrids shifted by the passivation energy
    const int sg = M.sub[i] == 0 ? 1 : -1;
    if (M.par.passivation_eV != 0.0) {
        for (int b = 0; b < 4; ++b) {
            if (M.nbr[i * 4 + b] >= 0) continue;
            double h[10] = {0};
            h[0] = 0.5;
            for (int a = 0; a < 3; ++a) h[1 + a] = 0.5 * sg * kSlot[b][a];
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) D0[r * nb + c] += M.par.passivation_eV * h[r] * h[c];
        }
    }
    for (int k = 0; k < no * no; ++k) D[k] = 0.0;
    for (int sp = 0; sp < (M.spin ? 2 : 1); ++sp)
        for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c) D[(sp * nb + r) * no + sp * nb + c] = D0[r * nb + c];
    if (M.spin) {
        // lambda L.S on the p shell, lambda = 2 Delta / 3, spin-major basis:
        // [[L_z, L_x - i L_y], [L_x + i L_y, -L_z]] * lambda / 2 with
        // (L_k)_{ab} = -i eps_{kab} on (px, py, pz).
        const double lam = 2.0 * M.so_par[sp_i] / 3.0;
        const cplx I(0.0, 1.0);
        cplx L[3][3][3];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    int e = 0;
                    if (a != b && a != k && b != k) e = ((a - k + 3) % 3 == 1) ? 1 : -1;
                    L[k][a][b] = -I * double(e);
                }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const int ra = 1 + a, cb = 1 + b;
                D[ra * no + cb] += 0.5 * lam * L[2][a][b];
                D[(nb + ra) * no + nb + cb] -= 0.5 * lam * L[2][a][b];
                D[ra * no + nb + cb] += 0.5 * lam * (L[0][a][b] - I * L[1][a][b]);
                D[(nb + ra) * no + cb] += 0.5 * lam * (L[0][a][b] + I * L[1][a][b]);
            }
    }
    // bonds: A atoms compute; B atoms take the conjugate transpose of the
    // partner's block so that H is Hermitian bit for bit
    cplx tmp[400];
    for (int b = 0; b < 4; ++b) {
        cplx* out = B + size_t(b) * no * no;
        const int64_t j = M.nbr[i * 4 + b];
        if (j < 0) {
            for (int k = 0; k < no * no; ++k) out[k] = 0.0;
            continue;
        }
        if (M.sub[i] == 0) {
            a_bond_block(M, i, b, out);
        } else {
            a_bond_block(M, j, b, tmp);
            for (int r = 0; r < no; ++r)
                for (int c = 0; c < no; ++c) out[r * no + c] = std::conj(tmp[c * no + r]);
        }
    }
}

Layout make_layout(int64_t n_atoms, int n_o, bool cplx_h, int prec, int R, bool diag) {
    Layout L;
    L.n_o = n_o;
    L.R = R;
    L.G = n_o / R;
    L.A = 64 / L.G;
    L.L = L.A * L.G;
    L.cs = cplx_h ? 2 : 1;
    L.esz = prec == TBH_F64 ? 8 : 4;
    L.K = 16 / L.esz;
    L.bond_chunks = (R * n_o * L.cs + L.K - 1) / L.K;
    L.onsite_chunks = ((diag ? R : R * n_o * L.cs) + L.K - 1) / L.K;
    L.C = 4 * L.bond_chunks + L.onsite_chunks;
    L.diag = diag;
    L.n_tiles = (n_atoms + L.A - 1) / L.A;
    L.bytes = L.n_tiles * int64_t(L.C) * L.L * 16;
    return L;
}

Layout make_layout_sd(int64_t n_atoms, int n_o, int prec, int R) {
    Layout L;
    const int nb = n_o / 2;
    L.sd = true;
    L.n_o = n_o;
    L.R = R;
    L.G = nb / R;
    L.A = 64 / L.G;
    L.L = L.A * L.G;
    L.cs = 2;
    L.esz = prec == TBH_F64 ? 8 : 4;
    L.K = 16 / L.esz;
    L.bond_chunks = (R * nb + L.K - 1) / L.K;
    L.onsite_chunks = (2 * R * n_o * 2 + L.K - 1) / L.K;
    L.C = 4 * L.bond_chunks + L.onsite_chunks;
    L.diag = false;
    L.n_tiles = (n_atoms + L.A - 1) / L.A;
    L.bytes = L.n_tiles * int64_t(L.C) * L.L * 16;
    return L;
}

namespace {

// spin-diagonal packing: per bond the real orbital block b of I_2 (x) b, then
// the full complex on-site rows of both spins; every bond block is checked
// for that form
template <typename T>
void pack_range_sd(const HostModel& M, const Layout& L, T* dst, int64_t t0, int64_t t1, const int64_t* perm) {
    const int no = M.n_o, nb = no / 2;
    std::vector<cplx> D(no * no), B(4 * no * no);
    for (int64_t t = t0; t < t1; ++t) {
        for (int la = 0; la < L.A; ++la) {
            const int64_t a = t * L.A + la;
            const bool live = a < M.n;
            if (live) {
                host_atom_blocks(M, perm ? perm[a] : a, D.data(), B.data());
                for (int b = 0; b < 4; ++b)
                    for (int r = 0; r < no; ++r)
                        for (int c = 0; c < no; ++c) {
                            const cplx v = B[(size_t(b) * no + r) * no + c];
                            const cplx want = (r / nb == c / nb) ? B[(size_t(b) * no + r % nb) * no + c % nb] : 0.0;
                            TBH_REQUIRE(v.imag() == 0.0 && v == want,
                                        "spin-diagonal storage needs every bond block to be I_2 (x) a real block");
                        }
            }
            for (int g = 0; g < L.G; ++g) {
                const int lane = la * L.G + g;
                auto put = [&](int s, double v) {
                    const int c = s / L.K, e = s % L.K;
                    dst[((t * L.C + c) * L.L + lane) * L.K + e] = live ? T(v) : T(0);
                };
                for (int b = 0; b < 4; ++b) {
                    const int base = b * L.bond_chunks * L.K;
                    int s = 0;
                    for (int r = 0; r < L.R; ++r)
                        for (int c = 0; c < nb; ++c) put(base + s++, B[(size_t(b) * no + g * L.R + r) * no + c].real());
                    while (s < L.bond_chunks * L.K) put(base + s++, 0.0);
                }
                const int base = 4 * L.bond_chunks * L.K;
                int s = 0;
                for (int sp = 0; sp < 2; ++sp)
                    for (int r = 0; r < L.R; ++r)
                        for (int c = 0; c < no; ++c) {
                            const cplx v = D[(sp * nb + g * L.R + r) * no + c];
                            put(base + s++, v.real());
                            put(base + s++, v.imag());
                        }
                while (s < L.onsite_chunks * L.K) put(base + s++, 0.0);
            }
        }
    }
}

template <typename T>
void pack_range(const HostModel& M, const Layout& L, bool diag, T* dst, int64_t t0, int64_t t1,
                const int64_t* perm) {
    if (L.sd) {
        pack_range_sd(M, L, dst, t0, t1, perm);
        return;
    }
    const int no = M.n_o;
    std::vector<cplx> D(no * no), B(4 * no * no);
    for (int64_t t = t0; t < t1; ++t) {
        for (int la = 0; la < L.A; ++la) {
            const int64_t a = t * L.A + la;
            const bool live = a < M.n;
            if (live) host_atom_blocks(M, perm ? perm[a] : a, D.data(), B.data());
            for (int g = 0; g < L.G; ++g) {
                const int lane = la * L.G + g;
                auto put = [&](int s, double v) {
                    const int c = s / L.K, e = s % L.K;
                    dst[((t * L.C + c) * L.L + lane) * L.K + e] = live ? T(v) : T(0);
                };
                for (int b = 0; b < 4; ++b) {
                    const int base = b * L.bond_chunks * L.K;
                    int s = 0;
                    for (int r = 0; r < L.R; ++r)
                        for (int c = 0; c < no; ++c) {
                            const cplx v = B[(size_t(b) * no + g * L.R + r) * no + c];
                            put(base + s++, v.real());
                            if (L.cs == 2) put(base + s++, v.imag());
                        }
                    while (s < L.bond_chunks * L.K) put(base + s++, 0.0);
                }
                const int base = 4 * L.bond_chunks * L.K;
                int s = 0;
                if (diag) {
                    for (int r = 0; r < L.R; ++r) {
                        const int row = g * L.R + r;
                        put(base + s++, D[row * no + row].real());
                    }
                } else {
                    for (int r = 0; r < L.R; ++r)
                        for (int c = 0; c < no; ++c) {
                            const cplx v = D[(g * L.R + r) * no + c];
                            put(base + s++, v.real());
                            if (L.cs == 2) put(base + s++, v.imag());
                        }
                }
                while (s < L.onsite_chunks * L.K) put(base + s++, 0.0);
            }
        }
    }
}

}  // namespace

std::vector<int64_t> locality_order(const int32_t* q, int64_t n) {
    // Rows of conventional cells (z, y) in order; within a row, the atoms of
    // each diamond basis class (position mod 4) as a run along x.  The
    // neighbours of such a run in any one bond direction are one fixed class
    // of the other sublattice in the same or an adjacent row, one cell
    // offset away: again a run of consecutive atoms.  A wavefront's neighbour
    // gathers then read contiguous rows, and the rows it needs lie within one
    // row of cells of its own, so an XCD's L2 holds them.
    auto key = [&](int64_t i) {
        const int32_t* p = q + 3 * i;
        const int cls = ((p[0] & 3) * 4 + (p[1] & 3)) * 4 + (p[2] & 3);
        return std::array<int64_t, 4>{p[2] >> 2, p[1] >> 2, cls, p[0] >> 2};
    };
    std::vector<int64_t> perm(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) perm[size_t(i)] = i;
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
    for (int64_t i = 0; i < n; ++i)
        if (perm[size_t(i)] != i) return perm;
    return {};
}

void tabulate(const HostModel& M, const int64_t* perm, std::vector<double>& table, int& nu,
              std::vector<uint8_t>& keys) {
    const int no = M.n_o;
    const int ns = int(M.onsite_par.size() / 4);
    TBH_REQUIRE(!M.cplx_h && !M.spin, "tabulated blocks need a real H at Gamma without spin");
    TBH_REQUIRE(M.bond_scale.empty(), "tabulated blocks need unstrained bonds (no bond_scale)");
    TBH_REQUIRE(!(M.par.passivation_eV != 0.0 && M.n_dangling > 0),
                "tabulated blocks need diagonal on-site blocks (no passivation)");
    TBH_REQUIRE(ns >= 1 && ns <= 4, "tabulated blocks support at most 4 species");
    // key of a bond slot: (sublattice, species of the atom, species of the
    // neighbour, slot); every atom's blocks are checked against the first
    // block seen under its key, in parallel with per-thread tables
    constexpr int NK = 2 * 4 * 4 * 4;
    const size_t bsz = size_t(no) * no;
    HostModel M0 = M;
    M0.pot.clear();   // the potential is applied per atom by the kernel
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    if (M.n < 4096) nt = 1;
    struct Local {
        std::vector<double> blk, diag;
        std::vector<char> has, has_d;
        bool bad = false;
        std::string why;
    };
    std::vector<Local> loc(nt);
    auto work = [&](unsigned w, int64_t a0, int64_t a1) {
        Local& L = loc[w];
        L.blk.assign(NK * bsz, 0.0);
        L.has.assign(NK, 0);
        L.diag.assign(size_t(ns) * no, 0.0);
        L.has_d.assign(ns, 0);
        std::vector<cplx> D(bsz), B(4 * bsz);
        for (int64_t i = a0; i < a1 && !L.bad; ++i) {
            host_atom_blocks(M0, i, D.data(), B.data());
            const int si = M.species[i];
            for (int r = 0; r < no; ++r)
                for (int c = 0; c < no; ++c) {
                    const double v = D[size_t(r) * no + c].real();
                    if (r != c) {
                        if (v != 0.0) {
                            L.bad = true;
                            L.why = "an on-site block is not diagonal";
                        }
                    } else if (!L.has_d[si]) {
                        L.diag[size_t(si) * no + r] = v;
                    } else if (L.diag[size_t(si) * no + r] != v) {
                        L.bad = true;
                        L.why = "on-site energies differ between atoms of one species";
                    }
                }
            L.has_d[si] = 1;
            for (int b = 0; b < 4; ++b) {
                const int32_t j = M.nbr[size_t(i) * 4 + b];
                if (j < 0) continue;
                const int kid = ((M.sub[i] * 4 + si) * 4 + M.species[j]) * 4 + b;
                double* t = &L.blk[size_t(kid) * bsz];
                const cplx* src = &B[size_t(b) * bsz];
                if (!L.has[kid]) {
                    for (size_t e = 0; e < bsz; ++e) t[e] = src[e].real();
                    L.has[kid] = 1;
                } else {
                    for (size_t e = 0; e < bsz; ++e)
                        if (t[e] != src[e].real()) {
                            L.bad = true;
                            L.why = "bond blocks are not determined by (sublattice, species pair, slot)";
                            break;
                        }
                }
            }
        }
    };
    {
        std::vector<std::thread> th;
        const int64_t per = (M.n + nt - 1) / nt;
        for (unsigned w = 0; w < nt; ++w) {
            const int64_t a0 = w * per, a1 = std::min<int64_t>(M.n, a0 + per);
            th.emplace_back(work, w, a0, std::max(a0, a1));
        }
        for (auto& t : th) t.join();
    }
    // merge, checking that the threads agree
    std::vector<double> blk(NK * bsz, 0.0), diag(size_t(ns) * no, 0.0);
    std::vector<char> has(NK, 0), has_d(ns, 0);
    for (const Local& L : loc) {
        if (L.bad) throw Error(TBH_EINVAL, "tabulated blocks: " + L.why);
        for (int k = 0; k < NK; ++k) {
            if (!L.has[k]) continue;
            if (!has[k]) {
                std::copy(L.blk.begin() + k * bsz, L.blk.begin() + (k + 1) * bsz, blk.begin() + k * bsz);
                has[k] = 1;
            } else if (!std::equal(L.blk.begin() + k * bsz, L.blk.begin() + (k + 1) * bsz, blk.begin() + k * bsz)) {
                throw Error(TBH_EINVAL, "tabulated blocks: bond blocks are not determined by the key");
            }
        }
        for (int sp = 0; sp < ns; ++sp) {
            if (!L.has_d[sp]) continue;
            if (!has_d[sp]) {
                std::copy(L.diag.begin() + sp * no, L.diag.begin() + (sp + 1) * no, diag.begin() + sp * no);
                has_d[sp] = 1;
            } else if (!std::equal(L.diag.begin() + sp * no, L.diag.begin() + (sp + 1) * no, diag.begin() + sp * no)) {
                throw Error(TBH_EINVAL, "tabulated blocks: on-site energies differ within a species");
            }
        }
    }
    // dense table
    int dense[NK];
    nu = 0;
    for (int k = 0; k < NK; ++k) dense[k] = has[k] ? nu++ : -1;
    TBH_REQUIRE(nu <= 254, "too many distinct bond blocks");
    table.assign(size_t(nu) * bsz + size_t(ns) * no, 0.0);
    for (int k = 0; k < NK; ++k)
        if (has[k]) std::copy(blk.begin() + k * bsz, blk.begin() + (k + 1) * bsz, table.begin() + dense[k] * bsz);
    std::copy(diag.begin(), diag.end(), table.begin() + size_t(nu) * bsz);
    // key records in stream order
    keys.assign(size_t(M.n) * 8, 0);
    for (int64_t k = 0; k < M.n; ++k) {
        const int64_t i = perm ? perm[k] : k;
        uint8_t* r = &keys[size_t(k) * 8];
        for (int b = 0; b < 4; ++b) {
            const int32_t j = M.nbr[size_t(i) * 4 + b];
            r[b] = j < 0 ? 255 : uint8_t(dense[((M.sub[i] * 4 + M.species[i]) * 4 + M.species[j]) * 4 + b]);
        }
        r[4] = M.species[i];
    }
}

void pack_atom_major(const HostModel& M, int64_t stride, float* dst) {
    const int no = M.n_o;
    const int cs = M.cplx_h ? 2 : 1;
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    if (M.n < 1024) nt = 1;
    auto work = [&](int64_t a0, int64_t a1) {
        std::vector<cplx> D(no * no), B(4 * no * no);
        for (int64_t a = a0; a < a1; ++a) {
            host_atom_blocks(M, a, D.data(), B.data());
            float* o = dst + a * stride;
            int64_t s = 0;
            for (int k = 0; k < 4 * no * no; ++k) {
                o[s++] = float(B[k].real());
                if (cs == 2) o[s++] = float(B[k].imag());
            }
            for (int k = 0; k < no * no; ++k) {
                o[s++] = float(D[k].real());
                if (cs == 2) o[s++] = float(D[k].imag());
            }
            while (s < stride) o[s++] = 0.f;
        }
    };
    std::vector<std::thread> th;
    const int64_t per = (M.n + nt - 1) / nt;
    for (unsigned w = 0; w < nt; ++w) {
        const int64_t a0 = w * per, a1 = std::min<int64_t>(M.n, a0 + per);
        if (a0 < a1) th.emplace_back(work, a0, a1);
    }
    for (auto& t : th) t.join();
}

void pack_layout(const HostModel& M, const Layout& L, bool diag, void* dst, const int64_t* perm) {
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    if (L.n_tiles < 64) nt = 1;
    std::vector<std::thread> th;
    // a worker's error (a block that does not fit the layout) is rethrown here
    std::vector<std::exception_ptr> err(nt);
    const int64_t per = (L.n_tiles + nt - 1) / nt;
    for (unsigned w = 0; w < nt; ++w) {
        const int64_t t0 = w * per, t1 = std::min<int64_t>(L.n_tiles, t0 + per);
        if (t0 >= t1) break;
        th.emplace_back([&, w, t0, t1] {
            try {
                if (L.esz == 8) pack_range<double>(M, L, diag, static_cast<double*>(dst), t0, t1, perm);
                else pack_range<float>(M, L, diag, static_cast<float*>(dst), t0, t1, perm);
            } catch (...) {
                err[w] = std::current_exception();
            }
        });
    }
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

}  // namespace tbh
