// Internal declarations of libbem (host data structures, device buffers, kernels' launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <complex>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bem.h"

namespace bem {

using cd = std::complex<double>;

// Status-carrying exception used inside the library; converted to a status code at the ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define BEM_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::bem::Error(BEM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
constexpr double kEta0 = kMu0 * kC0;
// Near-pair factor: a hair below 2 so that structured meshes never sit exactly on the threshold.
constexpr double kNearFactor = 2.0 - 2e-9;
constexpr int kMaxValence = 16;

// ---------------------------------------------------------------- host mesh

struct Mesh {
  int64_t nv = 0, nt = 0, ne = 0, nobj = 0;
  std::vector<double> xyz;        // nv*3
  std::vector<int32_t> tri;       // nt*3
  std::vector<int32_t> obj;       // nt
  std::vector<int64_t> obj_tri;   // nobj+1: triangles of object o are [obj_tri[o], obj_tri[o+1])
  std::vector<int64_t> obj_edge;  // nobj+1: edges of object o (library order is grouped by object)
  // geometry per triangle
  std::vector<double> area, normal, centroid, hmax;  // nt, 3nt, 3nt, nt
  // edges (library order: by T+ then local index)
  std::vector<int32_t> ev;        // 2*ne, va < vb
  std::vector<int32_t> tp, tm;    // T+, T-
  std::vector<int8_t> ip, im;     // local index of the free vertex in T+, T-
  std::vector<int32_t> tri_edge;  // 3*nt: edge opposite local vertex i
  std::vector<int8_t> tri_sign;   // 3*nt: +1 if the triangle is T+ of that edge
  // vertex fans: for vertex v, triangles and edges in cyclic order
  std::vector<int64_t> vptr;      // nv+1, CSR over incident edges (= valence)
  std::vector<int32_t> vedge;     // incident edges E_0..E_{N-1} in cyclic order
  std::vector<int32_t> vtri;      // triangle T_{k+1} lying between E_k and E_{k+1}
  int max_valence = 0;
  // near pairs (CSR over test triangles, sorted source lists)
  std::vector<int64_t> near_ptr;
  std::vector<int32_t> near_idx;
  // per object: the first object of which it is a translated copy (itself if none)
  std::vector<int32_t> geo_proto;
};

// Validates and builds the topology; throws Error(BEM_E_MESH, ...) on invalid input.
std::unique_ptr<Mesh> build_mesh(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                                 const int32_t* obj);

// Buffa-Christiansen data per dual cell, in the layout read by the K~ fill kernels.
// Cell v has N = valence(v) BC functions (its incident edges) and 2N sub-triangles
// in cyclic order.  Sub-triangle s of cell v: vertices v, m (edge midpoint), c
// (triangle centroid); stored relative to v.  The BC function b of cell v restricted
// to sub-triangle s is (alpha_b (r' - v) - beta_{b,s}) / (2 A_s).
struct CellData {
  int64_t ncell = 0;
  int maxv = 0;                     // padded valence
  std::vector<int32_t> nval;        // ncell
  std::vector<double> vpos;         // 3*ncell
  std::vector<double> sub_m, sub_c; // [slot][cell][3]  (slot < 2*maxv), relative to v
  std::vector<double> sub_area;     // [slot][cell]
  std::vector<int32_t> sub_parent;  // [slot][cell] primal triangle, -1 for padding
  std::vector<double> alpha;        // [b][cell]
  std::vector<double> beta;         // [b][slot][cell][3]
  std::vector<int64_t> col0;        // ncell: first column of the cell in its object's cell-expanded
                                    // K matrix (columns = (cell, BC) pairs of one object)
  std::vector<int64_t> obj_cell_ptr; // nobj+1, CSR of the cells (vertices) of every object
  std::vector<int32_t> obj_cells;
  std::vector<int64_t> obj_ncol;    // nobj: column count of each object's cell-expanded matrix
  std::vector<int64_t> colS, colT;  // per edge: its object-local columns in the cells of vs and vt
};
CellData build_cells(const Mesh& m);

// Near (T, v) pairs for the K~ fill: some triangle of the dual cell of v is near T.
void near_cells(const Mesh& m, std::vector<int64_t>& ptr, std::vector<int32_t>& idx);

}  // namespace bem
