// Host-side data structures shared by the C++ host sources and the HIP
// sources of the library (not part of the public ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "lfltsmc.h"

namespace lts {

constexpr int kLineKlTerms = LTS_LINE_KL_TERMS;

// A level on the host: the rectilinear grid, per-cell data, and the derived
// per-node data of the mass-lumped P1 discretization.
struct HostLevel {
  int nxc = 0, nyc = 0, nxn = 0, nyn = 0;
  std::vector<double> x, y;                 // node coordinates
  std::vector<uint8_t> active, fine, qoi;   // per cell
  std::vector<int32_t> block;               // per cell, -1 if inactive
  std::vector<uint8_t> flags;               // per node, LTS_NODE_* bits
  std::vector<double> mass, qoiw;           // per node
  int n_blocks = 0;
  double h = 0.0;
  int p = 1;
  double nu = 0.0;
  int n_dof = 0, n_P = 0, n_F = 0;
  // stabilized Chebyshev constants (Sec. 3.3); beta[k], beta_half[k] for k = 1..p-1
  double delta = 1.0, omega = 2.0;
  std::vector<double> beta, beta_half;
};

// Validates `d` and fills `out`; returns an error text ("" on success).
std::string build_level_from_desc(const lts_grid_desc& d, HostLevel& out);

// Generates the arrays of a rule-described level; returns "" on success.
std::string build_rect_desc(const lts_rect_rule& r, std::vector<double>& x, std::vector<double>& y,
                            std::vector<uint8_t>& active, std::vector<int32_t>& block,
                            std::vector<uint8_t>& fine, std::vector<uint8_t>& qoi, double& h,
                            int& p, int& n_blocks);

// Stabilized Chebyshev constants for (p, nu).
void cheb_constants(int p, double nu, double& delta, double& omega, std::vector<double>& beta,
                    std::vector<double>& beta_half);

// Per-sample substep coefficients for a step dt: out[0] = a_p (the
// coefficient of w after p substeps on a DOF outside F+), out[1] = c_1 (first
// substep), out[1+m] = c_2,m for m = 1..p-1.  Length p+1.
void step_coefficients(const HostLevel& L, double dt, double* out);

// Philox4x64-10 (Salmon et al., SC'11).
void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

// u[0..n-1]: uniforms ((x >> 12) + 0.5) 2^-52 of the stream with key (seed, 0)
// and counters (j, i, level, purpose), four per block j = 0, 1, ...
void philox_uniforms(uint64_t seed, int64_t i, int32_t level, uint64_t purpose, int n, double* u);

// A one-dimensional level (Sec. 4.1, 4.2): nodes, fine cells, lumped masses,
// the projector P and the stabilized Chebyshev constants.
struct LineHost {
  std::vector<double> x;        // nodes
  std::vector<uint8_t> fine;    // per cell
  std::vector<double> mass;     // per node
  std::vector<uint8_t> P;       // per node
  double H = 0.0;
  int p = 1;
  double nu = 0.0;
  int f0 = 0, nf = 0;           // F+ = nodes f0 .. f0+nf-1 (P and its neighbours; contiguous)
  double delta = 1.0, omega = 2.0;
  std::vector<double> beta, beta_half;
};

// Builds the level of `r`; "" on success.
std::string build_line_level(const lts_line_rule& r, LineHost& L);

// Per-sample cell coefficients kappa = c^2 [n][cells], step counts and dt for
// samples first .. first+n-1 of MLMC level sample_level on level L.
std::string gen_line_samples(uint64_t seed, int32_t sample_level, int64_t first, int32_t n,
                             const lts_line_sample_rule& rule, const LineHost& L, double* kappa,
                             int32_t* n_steps, double* dt);

std::string gen_samples(uint64_t seed, int32_t sample_level, int64_t first_index, int32_t n,
                        const lts_sample_rule& rule, double h_mesh, double* g, double* kappa,
                        double* x0, int32_t* n_steps, double* dt);

// A level given as a triangulation, built on the host.  DOFs are numbered
// in Morton order of their coordinates; the state of a sample holds the n_dof
// DOF values and a zero slot at index n_dof (the value of every Dirichlet
// neighbour).
constexpr int kTriRegionCap = LTS_MESH_REGION_CAP;
constexpr int kTriMaxDeg = LTS_MESH_MAX_DEGREE;
struct TriEnt {            // one node of a fine tile's region
  int32_t dof;             // DOF index | 0x80000000 if the DOF is in P
  int32_t row;             // first stiffness coupling of the DOF (CSR offset)
  int32_t deg_dist;        // number of couplings | graph distance to the tile << 16
  int32_t slot0;           // offset of the region slots of its couplings (tslot)
};
struct TriHost {
  HostLevel shell;                       // n_blocks, h, p, nu and the Chebyshev constants only
  int n_nodes = 0, n_tris = 0, n_dof = 0, n_P = 0, n_F = 0, max_deg = 0, max_region = 0;
  std::vector<int32_t> node_dof;         // [n_nodes] DOF index or -1
  std::vector<int32_t> dof_node;         // [n_dof]
  std::vector<double> mass_node;         // [n_nodes] lumped mass
  std::vector<uint8_t> node_flags;       // [n_nodes] LTS_NODE_* bits
  std::vector<double> dx, dy, invm, qoiw;   // [n_dof]
  std::vector<uint8_t> dflag;            // [n_dof + 1] bit 0: P, bit 1: F+ (the zero slot: 0)
  std::vector<int32_t> rp, col;          // CSR over the DOFs; col = n_dof for a Dirichlet neighbour
  std::vector<int32_t> eblk;             // block of the first | second triangle << 8 (255: none)
  std::vector<double> ewa, ewb;          // -|T| grad(l_i).grad(l_j) of those triangles (0: none)
  std::vector<int32_t> coarse;           // DOFs outside F+, increasing
  std::vector<int32_t> tiles;            // [n_tiles + 1] offsets of the tiles' regions in ent
  std::vector<TriEnt> ent;               // region nodes, tile by tile, by increasing distance
  std::vector<uint16_t> tslot;           // per region node and coupling: the neighbour's region
                                         // index if it is in P and in the region, else the region size
  double halo_ratio = 1.0;
};

// Validates `d` and builds T; "" on success.
std::string build_tri(const lts_mesh_desc& d, TriHost& T);

// Cost model of one solve in DOF updates: ceil(T/(cfl h)) ((N - |P|) + p |P|).
double solve_cost_model(const HostLevel& L, const lts_sample_rule& rule);

}  // namespace lts
