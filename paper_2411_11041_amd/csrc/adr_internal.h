// Internal declarations of the directional diffusion splitting library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/adr.h"

namespace adr {

// Error carrier used inside the library; converted to adr_status at the ABI.
struct Error {
    adr_status code;
    std::string msg;
};

// Rectangular mesh over the bounding box (eq. (20)).
struct Grid {
    double a, b, c, d, hx, hy, h;
    int nx, ny;
    double x(int i) const { return a + hx * i; }
    double y(int j) const { return c + hy * j; }
    // eq. (21)/(23): 0-based floor clamped to the last cell, y index from y.
    void cell(double px, double py, int &i, int &j, double &lx, double &ly) const;
    // eq. (22): bilinear value of a nodal field.
    double interp(const double *F, double px, double py) const;
};

// One traced family of curves (polylines).
struct Family {
    std::vector<int64_t> off;   // line l: nodes off[l] .. off[l+1]-1
    std::vector<double> x, y;
};

// The scatter stencil of one grid node: value = gb + sum over the 4 records of
// ca * v[k] + cb * v[k+1] (k = -1: unused); gb = the Dirichlet data its
// boundary points carry (0 for zero data).
struct Rec4 {
    int32_t k[4];
    double ca[4], cb[4];
    double gb;
    // the same stencil factored (records 0, 1 horizontal, 2, 3 vertical):
    // ca[r] = W_r lam_r (1 - t[r]), cb[r] = W_r lam_r t[r] with W = (wh, wh, 1 - wh, 1 - wh)
    // and lam = (lam[0], 1 - lam[0], lam[1], 1 - lam[1]); t = 0 at boundary points
    double wh, lam[2], t[4];
};

// Everything the device needs for one instance, in local indices.
// The interpolation-free transfer onto one interior node of a target curve:
// value = (k[0] >= 0 ? w[0] v[k[0]] + w[1] v[k[0]+1] : w[0] x_first)
//       + (k[1] >= 0 ? w[2] v[k[1]] + w[3] v[k[1]+1] : w[2] x_last)
// with v the other family's line values (k: first node of the source segment
// of the bracket; -1: the target curve's own end on that side, whose
// Dirichlet value x_first or x_last it carries).
struct DirRec {
    int32_t k[2];
    double w[4];
};

struct InstanceGeo {
    Grid g;
    double mu, sigma;
    std::vector<uint8_t> inner;        // nx*ny interior-node mask
    std::vector<int32_t> inner_list;   // local grid indices of interior nodes
    Family fam[2];
    // per family, per node
    std::vector<double> hk[2];         // chord to the previous node (0 at a line start)
    std::vector<int32_t> cellk[2];     // bottom-left corner (local grid index), -1 at line ends
    std::vector<double> lxk[2], lyk[2];
    std::vector<double> wk;            // beta family: |beta| at the node
    std::vector<double> Lk;            // beta family: load int f phi_k (0 at ends)
    std::vector<Rec4> rec[2];          // per interior node (inner_list order)
    std::vector<DirRec> drec[2];       // direct transfer onto family f's nodes (options.transfer = 1)
    std::vector<double> gend[2];       // per curve: Dirichlet data at its first and last node
    bool has_g = false;                // non-zero Dirichlet data given
};

// Message returned by adr_last_error(NULL) in this thread (failed set-up or
// context-free call).
void set_thread_error(const std::string &msg);

// Direct-transfer records of every node of tgt (interior nodes; ends unused)
// from the line values of src; htgt: tgt's chords (hk).
void build_direct(const Grid &g, const Family &tgt, const std::vector<double> &htgt, const Family &src,
                  std::vector<DirRec> &out);

// Builds the geometry of one instance; throws Error.
void build_instance(const adr_problem &p, InstanceGeo &out);
// Load vector of the beta-curves for the source of p (curves already traced).
void compute_load(const adr_problem &p, InstanceGeo &G);
// Load vector of a traced beta family for the nodal source f (chords from the nodes).
void load_from_positions(const Grid &g, const Family &F, const double *f, std::vector<double> &L);
// Copy of base (same grid, domain and beta) with the coefficients and source of p.
void rebuild_for_source(const InstanceGeo &base, const adr_problem &p, InstanceGeo &out);

}  // namespace adr
