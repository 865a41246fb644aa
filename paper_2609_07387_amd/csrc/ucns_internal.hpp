// Internal host-side structures of libucns (not part of the C ABI).
#pragma once
#include <cstddef>
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ucns.h"

namespace ucns {

constexpr int kMaxFaces = 6;     // faces per cell
constexpr int kMaxQ = 16;         // quadrature points per face (4x4 at P4)
constexpr int kMaxK = 34;         // unknowns at P4
constexpr int kMaxKd = 9;         // unknowns of a directional polynomial (quadratic at P4)
constexpr int kMaxCentral = 128;  // central stencil cap
constexpr int kMaxDir = 32;       // directional stencil cap
// Directional stencils of a polynomial with kd unknowns: the 2 (kd + 1)
// nearest sector candidates before closure (8 linear, 20 quadratic); fewer
// than kd + 1 drop the sector (4 linear, 10 quadratic).
inline int dir_target(int kd) { return 2 * (kd + 1); }
inline int dir_min(int kd) { return kd + 1; }
constexpr int kNumVar = 5;

void set_error(const std::string& msg);

// Point states are stored per point slot (lf, q) as a row of [cell][5]
// values, the cell count padded to whole 64-cell tiles (a wave stages its 64
// cells' values and writes the tile's 320 values as five contiguous runs).
constexpr int64_t kFsTile = 64;
constexpr int64_t fs_cells_padded(int64_t nc) { return (nc + kFsTile - 1) / kFsTile * kFsTile; }

// Largest byte span one buffer descriptor of the reconstruction kernels
// covers (offsets inside a descriptor are 32-bit, so it must stay below
// 4 GiB): the state U (5 rows of FP64), a member's or the basis means' K
// operator rows, or the NF rows of face-neighbour ids.  Every other stream
// (stencil ids, face-point offsets, directional operators, point states)
// takes its row index in the descriptor's 64-bit base and spans at most
// 5 rows of the precision's type (a point-state slot: 5 values per cell of
// the padded count).
inline uint64_t recon_span_bytes(int64_t nc, int elem_bytes, int K, int NF) {
    uint64_t per_cell = 40;
    per_cell = std::max<uint64_t>(per_cell, uint64_t(K) * uint64_t(elem_bytes));
    per_cell = std::max<uint64_t>(per_cell, uint64_t(NF) * 4u);
    return std::max<uint64_t>(per_cell * uint64_t(nc),
                              uint64_t(5) * uint64_t(elem_bytes) * uint64_t(fs_cells_padded(nc)));
}
constexpr uint64_t kMaxDescriptorBytes = 0xffffffffull;


// Offsets (bytes) of every array inside one precision's device arena.
struct Arena {
    size_t bytes = 0;
    size_t sten_c = 0, Bc = 0, ndir = 0, sten_d = 0, Bd = 0, O = 0, xi = 0, pmean = 0, c2f = 0;
    size_t cnq = 0;  // [nfmax][nc] Gauss points of each of a cell's face slots (0: no face)
    size_t vol = 0, hdt = 0, fcell = 0, flf = 0, fnrm = 0, farea = 0, fw = 0, fdc = 0, fnq = 0;
    // face neighbours ([nfmax][nc]; a boundary slot holds its face's negative tag, an absent one -1),
    // their centroid offsets, basis scale, stencil size (gate features; fused gradients)
    size_t nbr = 0, ndc = 0, hb = 0, ncen = 0;
    size_t glsq = 0;  // [nfmax][3][nc] least-squares gradient weights per face slot
    size_t ggw = 0;   // [nfmax][3][nc] Green-Gauss weights per face slot: outward n |S| / (2 |V|)
    size_t ustage = 0;  // P4 only: [nc][8] FP64, the state staged cell-interleaved by each reconstruction call
    void* dev = nullptr;  // caller-owned device pointer after upload
};

struct Mesh {
    // ---- input
    int64_t nv = 0, nc = 0;
    std::vector<double> xyz;
    std::vector<uint8_t> type;
    std::vector<int64_t> cptr, cvtx;
    double period[3] = {0, 0, 0};
    // ---- options
    int order = 2, K = 9, qmax = 4, nfmax = 6, max_layers = 3;
    int kd = 3;  // unknowns of the directional polynomials: 3 (linear, P2/P3), 9 (quadratic, P4)
    bool uniform_type = true;  // every cell of one type
    double lambda_c = 1000.0, eps = 1e-12;
    double stencil_factor = 2.0;  // central stencil = round(stencil_factor K(r,3)) cells
    // ---- faces (numbered by owner cell, then owner-local face)
    int64_t nf = 0, nbnd = 0;
    std::vector<int64_t> fcell;   // [nf][2]; side 1 = -1 - tag on the boundary
    std::vector<int> flf;         // [nf][2] local face indices
    std::vector<int> fnq;         // points per face
    std::vector<double> farea, fnrm, fqp, fqw, fshift, fcen, fdc;  // fdc: owner->neighbour centroid offset
    std::vector<int32_t> c2f;     // [nc][kMaxFaces] = 2 f + side, -1 unused
    // ---- cells
    std::vector<double> vol, cen, hb, hdt;
    std::vector<double> glsq;     // [nc][kMaxFaces][3] least-squares gradient weights
    double total_vol = 0;  // sum of vol, in cell order
    std::vector<double> moments;  // [nc][nmom] central moments
    int mom_deg = 0, nmom = 0;
    // ---- stencils
    std::vector<int> ncen, navail;
    std::vector<int64_t> cand;    // [nc][kMaxCentral] sorted candidates
    std::vector<double> cdist;    // [nc][kMaxCentral]
    std::vector<int> ndir, ndropped;
    std::vector<int> nds, dface;  // [nc][kMaxFaces]
    std::vector<int64_t> dir;     // [nc][kMaxFaces][kMaxDir]
    int mc_pad = 0, md_pad = 0, nd_max = 0, mc_min = 0;
    // ---- operators (FP64, cell-major, for packing and inspection)
    std::vector<double> Bc;       // [nc][K][mc_pad]
    std::vector<double> Bd;       // [nc][nd_max][kd][md_pad]
    std::vector<double> O;        // [nc][K][K]
    std::vector<double> Phi;      // [nc][nfmax][qmax][K]
    std::vector<double> xi;       // [nc][nfmax][qmax][3] face points in the cell's scaled frame
    std::vector<double> mean;     // [nc][K]
    // ---- device arenas
    Arena arena[2];
    int64_t n_dropped_total = 0;
};

int build_mesh(const ucns_mesh_desc* d, const ucns_recon_opts* o, int n_threads, Mesh** out);
// Packs the arrays of one precision into a host image of the device arena.
int pack_arena(const Mesh& m, int precision, Arena& a, std::vector<unsigned char>* image);

int cell_nfaces(int type);
const int* face_verts(int type, int lf, int* nv);

}  // namespace ucns

struct ucns_mesh {
    ucns::Mesh* m;
};
