// Host-side preprocessed mesh: every array the device kernels read, in the
// library's internal numbering (cells on a Morton curve of their centres).
#pragma once
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace mifvm {

struct NnTiles;

// Rows packed in slices of 64 (one wavefront): slice s stores entry k of row
// 64*s + lane at off[s] + k*64 + lane, for k < width[s].  Short rows are
// padded with entries that contribute exactly zero (documented per use).
struct Sell64 {
    int64_t nslices = 0;
    std::vector<int64_t> off;      // nslices + 1
    std::vector<int32_t> width;    // nslices
    std::vector<int32_t> idx;      // off[nslices]
    std::vector<double> val;       // off[nslices] (empty when unused)
};

struct Mesh {
    int64_t nc = 0, nv = 0, nf = 0, nfi = 0, nb = 0;
    // independent meshes of a batch: internal cells [mesh_start[m], mesh_start[m+1])
    std::vector<int64_t> mesh_start;
    std::vector<int32_t> cell_perm;   // internal cell -> user cell
    std::vector<int32_t> vert_perm;   // internal vertex -> user vertex
    std::vector<double> vol;          // nc
    std::vector<double> xc;           // 3 x (nc+nb), SoA
    std::vector<double> minv;         // 6 x nc: xx xy xz yy yz zz
    // faces: interior [0,nfi), boundary [nfi,nf); boundary face nfi+g <-> ghost g
    std::vector<int32_t> fL, fR;      // R = nc+g on the boundary
    std::vector<int32_t> fA, fB, fC;  // internal vertex ids
    std::vector<double> kAC, kBC, kRL;
    std::vector<double> fx;           // 3 x nf face centroid
    std::vector<double> S;            // 3 x nf face vector
    std::vector<double> area;         // nf
    // ghosts
    std::vector<int32_t> gowner, gtag;
    std::vector<double> gdist;
    std::vector<int32_t> gbtri;       // ghost -> index of the caller's boundary triangle
    // cell -> faces (f if the cell is L, ~f if R) and cell across each face
    std::vector<int32_t> c2f, c2n;    // 4 x nc
    // CSR forms (for export/tests) and packed forms (for the device)
    std::vector<int64_t> sptr; std::vector<int32_t> sidx;
    std::vector<int64_t> nptr; std::vector<int32_t> nidx; std::vector<double> nalpha;
    int32_t stencil_max = 0, node_max = 0, row_max = 0;
    int64_t matrix_nnz = 0;
    Sell64 stencil;                   // node-neighbour stencil, pad = the row itself
    Sell64 node;                      // vertex lists + weights, pad = first entry, weight 0
    Sell64 kmat;                      // Poisson off-diagonal pattern, pad = the row itself
                                      // (empty when preprocessed with no_matrix)
    std::vector<int32_t> klen;        // off-diagonal entries per row (sorted prefix)
    // Tiles of `tile_rows` consecutive cells (a multiple of 64).  Each tile's
    // halo is the sorted set of cells and ghosts its stencils reference
    // (its own cells included, contiguous); kernels stage the halo's data in
    // LDS and address it with 16-bit local indices laid out like the
    // corresponding 64-row slices.
    int32_t tile_rows = 256;
    int32_t halo_max = 0;
    std::vector<int64_t> h_off;       // ntiles + 1
    std::vector<int32_t> h_idx;       // halo entities
    std::vector<int32_t> h_self;      // ntiles: local index of the tile's first cell
    std::vector<uint16_t> k_lidx;     // like kmat.idx, local
    std::vector<uint16_t> c2n_l;      // 4 x nc local index of the face neighbour
    // vertices are numbered by their lowest cell, so the vertices of tile t
    // (those whose lowest cell lies in it) are [v_off[t], v_off[t+1]); their
    // cell/ghost lists lie inside the tile's halo
    std::vector<int64_t> v_off;       // ntiles + 1
    std::vector<uint16_t> n_lidx;     // like node.idx, local to the owning tile
    // Star-moment form of the gradient sum of Algorithm 1.  An entity of the
    // stencil of cell i shares m in {1, 2, 3} vertices with i, so the sum
    // over the stencil equals the sum over the 4 vertex lists of i minus
    // (m - 1) times each entity with m > 1: the entities sharing exactly an
    // edge (m = 2, listed here) and the 4 face neighbours (m = 3, c2n).
    std::vector<int64_t> eptr; std::vector<int32_t> eidx;   // edge-only neighbours, CSR
    Sell64 enbr;                      // the same, pad = the row itself
    std::vector<uint16_t> e_lidx;     // like enbr.idx, local to the tile
    int32_t enbr_max = 0;
    std::vector<int32_t> n_len;       // nv: vertex list lengths
    // Vertices a tile's cells touch: the tile's own ([v_off[t], v_off[t+1]))
    // and the foreign ones, listed per tile with their vertex lists in the
    // tile's local halo indices (pad = first entry).  Tile-local vertex
    // number: own v -> v - v_off[t], foreign row r -> own count + r - fv_off[t].
    std::vector<int64_t> fv_off;      // ntiles + 1
    std::vector<int32_t> fv_idx;      // foreign vertex ids
    std::vector<int32_t> fv_len;      // their list lengths
    Sell64 fnode;                     // their lists, idx local (stored in f_lidx)
    std::vector<uint16_t> f_lidx;
    std::vector<uint16_t> c2v_l;      // 4 x nc tile-local vertex number
    int32_t tv_max = 0;               // most vertices touched by one tile
    // tiles of the network's fused forward, built on first use
    mutable std::shared_ptr<const NnTiles> nn_tiles;
};

// Returns 0 or a negative mifvm status; err receives a message.
// mesh_cell_start (nmeshes+1 entries, or null for one mesh) splits the tets
// into independent meshes; each must have at least 256 cells when nmeshes > 1.
int preprocess(const double* xyz, int64_t nv, const int32_t* tets, int64_t nc,
               const int32_t* btris, const int32_t* btags, int64_t nb,
               int renumber, const int64_t* mesh_cell_start, int32_t nmeshes, bool no_matrix, Mesh& out,
               std::string& err);

}  // namespace mifvm
