// Internal declarations of libpdg: host context, setup routines and kernel
// launchers.  Not part of the ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pdg.h"

namespace pdg {

struct Error : std::runtime_error {
    pdg_status code;
    Error(pdg_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

constexpr int kTile = 64;           // dense inverse tile edge
constexpr int kMaxLocalDofs = 6144;   // largest subdomain (dense inverse per subdomain)
constexpr int kMaxCoarseDofs = 16384; // largest coarse system per batch system (dense inverse, 2 GiB)
constexpr int kIonicParams = 24;
constexpr int kStates = 5;

// ---- host FEM (fem.cpp) ----------------------------------------------------
int n_basis(int dim, int p);
void multi_indices(int dim, int p, std::vector<int> &alpha);  // [nd][3] (unused dims 0)
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w);
// values (and derivatives) of the modal basis at reference point xi in [-1,1]^dim
void basis_eval(int dim, int p, const int *alpha, int nd, const double *xi, const double *ext,
                double *phi, double *dphi /* [nd][dim] or null */);
double lambda_max_sym(int dim, const double *S);

struct Mesh {
    int dim = 0, p = 0, nd = 0;
    int64_t n_elem = 0, n_facet = 0;
    std::vector<int64_t> cell_ptr, facet_elem;
    std::vector<double> cell_geom, facet_geom, facet_normal, sigma;
    std::vector<int> alpha;          // [nd][3]
    std::vector<double> lo, hi, hK;  // bbox [n_elem][dim], diameter
    // element quadrature in bbox reference coordinates
    std::vector<int64_t> qp_ptr;     // [n_elem+1]
    std::vector<double> qp_xi;       // [nq][dim]
    std::vector<double> qp_w;        // [nq]
    std::vector<double> norm;        // [n_elem][nd]: prod_j sqrt((2a_j+1)/ext_j)
};

struct Bsr {
    int64_t n_rows = 0, nnzb = 0;
    int nd = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val;  // [nnzb][nd][nd]
};

void build_mesh(Mesh &m, const pdg_mesh *in, int p);
// Mass blocks M [n_elem][nd][nd] and K = c M + 1/2 A in BSR.
void assemble(const Mesh &m, double c, double eta0, std::vector<double> &M, Bsr &K);
void element_inverse(int n, const double *A, double *Ainv);  // small SPD inverse (FP64)

// ---- dense SPD inversion and Schwarz setup (schwarz_setup.cpp) -------------
// In-place inverse of a dense SPD matrix (row-major n x n).  Throws ENOTSPD.
void spd_inverse(int64_t n, double *A, int n_threads = 1);

struct DenseSys {
    int64_t n = 0;          // true size
    int64_t nt = 0;         // tiles per edge
    int64_t tile_off = 0;   // offset (in tiles) into the tile store
};

// bfloat16 of v: v rounded to FP32, then to 8 significant bits (nearest, ties to even).
inline uint16_t bf16_bits(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
inline double bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

struct Precond {
    int n_sub = 0, n_coarse = 0, q = 0, nq0 = 0;
    int n_bsys = 1;                                // independent systems of the batch
    int local_prec = PDG_F64, coarse_prec = PDG_F64;
    std::vector<int32_t> sub_ptr, sub_elems;       // CSR of elements per subdomain
    std::vector<int32_t> sub_bsys;                 // batch system of each subdomain
    // coarse elements in internal numbering (those of one batch system contiguous)
    std::vector<int32_t> coarse_orig, cnum;        // internal -> caller label, caller label -> internal
    std::vector<int32_t> csys_ce0;                 // [n_bsys+1] first internal coarse element of each system
    std::vector<int32_t> coarse_ptr, coarse_elems; // CSR of elements per (internal) coarse element
    std::vector<int32_t> elem_coarse;              // internal coarse element of each element
    std::vector<DenseSys> sys;                     // n_sub local systems, then one coarse system per batch system
    std::vector<double> inv64;                     // FP64 inverse tiles (all systems)
    // BF16 local store: K_i^{-1} = D_i C_i D_i with D_i = diag(K_i^{-1})^{1/2}
    // (kept in FP32) and C_i (unit diagonal) rounded to BF16.  A C_i whose
    // rounded form fails the positive-definiteness check is stored in FP32.
    std::vector<uint16_t> tiles_b16;               // C_i tiles of the local systems (local tile offsets)
    std::vector<float> dscale;                     // d of every local system, nt * 64 rows each (0 past n)
    std::vector<int64_t> rbase;                    // [n_sub] first row of each local system in dscale
    std::vector<int32_t> fallback;                 // [n_sub] 1: stored in FP32
    int n_fallback = 0;
    int64_t n_tiles = 0;
    std::vector<double> P;                         // [n_elem][nd][nq0]
    std::vector<std::vector<double>> K0blk;        // K0 of each batch system, internal order
    int64_t N0 = 0;                                // coarse dofs over all systems
};

// elem_bsys: batch system of every element (all 0 for one system).
// bf16_margin: a BF16 local store keeps C_i only if C_i rounded to BF16,
// minus bf16_margin times the identity, is positive definite.
void setup_precond(const Mesh &m, const Bsr &K, const std::vector<double> &Mblk,
                   const pdg_precond_desc *d, const std::vector<int32_t> &elem_bsys, int n_bsys, Precond &pc,
                   int n_threads, double bf16_margin);
void dense_inverse_of_system(const Precond &pc, int s, std::vector<double> &out);

}  // namespace pdg
