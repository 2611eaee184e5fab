// Host preprocessing of an unstructured tetrahedral mesh for the
// cell-centred finite-volume kernels (the "readmesh + Domain" stage of the
// paper's annex, redesigned for one GPU holding the whole mesh).
//
// Geometry follows Sec. 2.1: data at cell centres of gravity, fluxes on
// faces with normal n_ij |sigma_ij|, ghost cells behind boundary faces, the
// node-neighbour stencil of Algorithm 1, the least-squares vertex weights of
// Algorithm 2, and the diamond cell of eq. (diamond) with a triangular base.
// Where the paper is silent this code takes the same readings as the rest
// of the library: ghost centre = owner centre mirrored across the face
// plane; an interior face's L cell is the owner with the smaller user index;
// vertex weights are the unweighted least-squares linear fit evaluated at
// the vertex; the gradient solves the 3x3 normal equations.
#include "mesh.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

namespace mifvm {
namespace {

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

uint64_t spread21(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

struct FaceRec {
    int32_t a, b, c;   // sorted user vertex ids
    int32_t owner;     // user cell id
};

// Solve the 4x4 system A w = rhs by Gaussian elimination with partial
// pivoting; returns false when singular.
bool solve4(double A[4][4], double rhs[4], double w[4]) {
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return false;
        if (piv != col) {
            for (int k = 0; k < 4; ++k) std::swap(A[col][k], A[piv][k]);
            std::swap(rhs[col], rhs[piv]);
        }
        for (int r = col + 1; r < 4; ++r) {
            double m = A[r][col] / A[col][col];
            for (int k = col; k < 4; ++k) A[r][k] -= m * A[col][k];
            rhs[r] -= m * rhs[col];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = rhs[r];
        for (int k = r + 1; k < 4; ++k) s -= A[r][k] * w[k];
        w[r] = s / A[r][r];
    }
    return true;
}

template <class PadIdx>
void pack_sell(const std::vector<int64_t>& ptr, const std::vector<int32_t>& idx,
               const std::vector<double>* val, const std::vector<int32_t>* len_override,
               int64_t nrows, PadIdx pad_idx, Sell64& out) {
    out.nslices = (nrows + 63) / 64;
    out.off.assign(out.nslices + 1, 0);
    out.width.assign(out.nslices, 0);
    auto rowlen = [&](int64_t r) -> int64_t {
        return len_override ? (*len_override)[r] : ptr[r + 1] - ptr[r];
    };
    for (int64_t s = 0; s < out.nslices; ++s) {
        int64_t w = 0;
        for (int64_t r = s * 64; r < std::min(nrows, s * 64 + 64); ++r) w = std::max(w, rowlen(r));
        out.width[s] = (int32_t)w;
        out.off[s + 1] = out.off[s] + w * 64;
    }
    out.idx.assign(out.off[out.nslices], 0);
    if (val) out.val.assign(out.off[out.nslices], 0.0);
    for (int64_t s = 0; s < out.nslices; ++s) {
        for (int lane = 0; lane < 64; ++lane) {
            int64_t r = s * 64 + lane;
            int64_t L = r < nrows ? rowlen(r) : 0;
            int32_t pad = r < nrows ? pad_idx(r) : 0;
            for (int64_t k = 0; k < out.width[s]; ++k) {
                int64_t at = out.off[s] + k * 64 + lane;
                if (k < L) {
                    out.idx[at] = idx[ptr[r] + k];
                    if (val) out.val[at] = (*val)[ptr[r] + k];
                } else {
                    out.idx[at] = pad;
                }
            }
        }
    }
}

}  // namespace

int preprocess(const double* xyz, int64_t nv, const int32_t* tets, int64_t nc,
               const int32_t* btris, const int32_t* btags, int64_t nb_in,
               int renumber, const int64_t* mesh_cell_start, int32_t nmeshes, bool no_matrix, Mesh& M,
               std::string& err) {
    const int E_ARG = -1, E_MESH = -2;
    if (!xyz || !tets || nv <= 0 || nc <= 0 || nb_in < 0 || (nb_in > 0 && (!btris || !btags))) {
        err = "null pointer or non-positive size";
        return E_ARG;
    }
    if (nc > (int64_t(1) << 30) || nv > (int64_t(1) << 30)) {
        err = "mesh too large for 32-bit indices";
        return E_ARG;
    }
    for (int64_t i = 0; i < 4 * nc; ++i)
        if (tets[i] < 0 || tets[i] >= nv) { err = "tet vertex index out of range"; return E_ARG; }
    for (int64_t i = 0; i < 3 * nb_in; ++i)
        if (btris[i] < 0 || btris[i] >= nv) { err = "boundary vertex index out of range"; return E_ARG; }
    for (int64_t i = 0; i < nb_in; ++i)
        if (btags[i] < 0 || btags[i] >= 32) { err = "boundary tag out of [0, 32)"; return E_ARG; }
    std::vector<int64_t> mstart = {0, nc};
    if (mesh_cell_start && nmeshes > 1) {
        if (nmeshes > 4096) { err = "too many meshes in one batch"; return E_ARG; }
        mstart.assign(mesh_cell_start, mesh_cell_start + nmeshes + 1);
        if (mstart[0] != 0 || mstart[nmeshes] != nc) { err = "mesh_cell_start must run from 0 to nc"; return E_ARG; }
        for (int32_t m = 0; m < nmeshes; ++m)
            if (mstart[m + 1] - mstart[m] < 256) { err = "every mesh of a batch needs at least 256 cells"; return E_ARG; }
    } else if (nmeshes > 1) {
        err = "mesh_cell_start is null";
        return E_ARG;
    }
    const int32_t nm = int32_t(mstart.size() - 1);
    std::vector<int32_t> mesh_of_user(nc);
    for (int32_t m = 0; m < nm; ++m)
        for (int64_t c = mstart[m]; c < mstart[m + 1]; ++c) mesh_of_user[c] = m;

    auto P = [&](int64_t v) { return V3{xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]}; };
    // MIFVM_PREPROCESS_TIMING=1 prints the time of each stage to stderr
    const bool timing = std::getenv("MIFVM_PREPROCESS_TIMING") != nullptr;
    auto tprev = std::chrono::steady_clock::now();
    auto mark = [&](const char* what) {
        if (!timing) return;
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[mifvm preprocess] %-28s %8.3f s\n", what,
                     std::chrono::duration<double>(now - tprev).count());
        tprev = now;
    };

    // -- 1. orientation, volume, centre of gravity (user order) --------------
    std::vector<std::array<int32_t, 4>> T(nc);
    std::vector<double> vol_u(nc);
    std::vector<V3> cen_u(nc);
    double vsum = 0;
    for (int64_t c = 0; c < nc; ++c) {
        std::array<int32_t, 4> t = {tets[4 * c], tets[4 * c + 1], tets[4 * c + 2], tets[4 * c + 3]};
        V3 p0 = P(t[0]), p1 = P(t[1]), p2 = P(t[2]), p3 = P(t[3]);
        double det = dot(sub(p1, p0), cross(sub(p2, p0), sub(p3, p0)));
        if (det < 0) std::swap(t[2], t[3]);
        T[c] = t;
        vol_u[c] = std::fabs(det) / 6.0;
        vsum += vol_u[c];
        V3 q0 = P(t[0]), q1 = P(t[1]), q2 = P(t[2]), q3 = P(t[3]);
        cen_u[c] = scale(add(add(add(q0, q1), q2), q3), 0.25);
    }
    double vmean = vsum / double(nc);
    for (int64_t c = 0; c < nc; ++c)
        if (!(vol_u[c] > 1e-14 * vmean)) { err = "degenerate tetrahedron"; return E_MESH; }

    mark("orientation+volumes");
    // -- 2. cell renumbering --------------------------------------------------
    std::vector<int32_t> new2old(nc), old2new(nc);
    std::iota(new2old.begin(), new2old.end(), 0);
    if (renumber == 1) {
        V3 lo = cen_u[0], hi = cen_u[0];
        for (auto& p : cen_u) {
            lo = {std::min(lo.x, p.x), std::min(lo.y, p.y), std::min(lo.z, p.z)};
            hi = {std::max(hi.x, p.x), std::max(hi.y, p.y), std::max(hi.z, p.z)};
        }
        double ext = std::max({hi.x - lo.x, hi.y - lo.y, hi.z - lo.z, 1e-300});
        double q = double((1 << 21) - 1) / ext;
        std::vector<uint64_t> key(nc);
        for (int64_t c = 0; c < nc; ++c) {
            auto cx = uint64_t((cen_u[c].x - lo.x) * q), cy = uint64_t((cen_u[c].y - lo.y) * q),
                 cz = uint64_t((cen_u[c].z - lo.z) * q);
            key[c] = spread21(cx) | (spread21(cy) << 1) | (spread21(cz) << 2);
        }
        // Morton order within each mesh; meshes stay contiguous and in order
        std::stable_sort(new2old.begin(), new2old.end(), [&](int32_t a, int32_t b) {
            if (mesh_of_user[a] != mesh_of_user[b]) return mesh_of_user[a] < mesh_of_user[b];
            return key[a] < key[b];
        });
    } else if (renumber == 2) {
        // Reverse Cuthill-McKee on the face-adjacency graph of the cells
        // (Cuthill & McKee 1969; reversed, George 1971), each mesh of a batch
        // and each connected component on its own: breadth-first from a
        // pseudo-peripheral cell (the George-Liu search: restart from the
        // lowest-degree cell of the last level until the depth stops
        // growing), neighbours visited by increasing degree then index, the
        // whole order reversed.
        std::vector<std::array<int32_t, 4>> key(4 * nc);
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < 4; ++k) {
                std::array<int32_t, 3> v = {T[c][(k + 1) % 4], T[c][(k + 2) % 4], T[c][(k + 3) % 4]};
                std::sort(v.begin(), v.end());
                key[4 * c + k] = {v[0], v[1], v[2], int32_t(c)};
            }
        std::sort(key.begin(), key.end());
        std::vector<int64_t> aptr(nc + 1, 0);
        std::vector<std::pair<int32_t, int32_t>> edges;
        for (size_t a = 0; a + 1 < key.size(); ++a)
            if (key[a][0] == key[a + 1][0] && key[a][1] == key[a + 1][1] && key[a][2] == key[a + 1][2])
                edges.emplace_back(key[a][3], key[a + 1][3]);
        key.clear();
        key.shrink_to_fit();
        for (auto& e : edges) { aptr[e.first + 1]++; aptr[e.second + 1]++; }
        for (int64_t c = 0; c < nc; ++c) aptr[c + 1] += aptr[c];
        std::vector<int32_t> adj(aptr[nc]);
        {
            std::vector<int64_t> pos(aptr.begin(), aptr.end() - 1);
            for (auto& e : edges) { adj[pos[e.first]++] = e.second; adj[pos[e.second]++] = e.first; }
        }
        edges.clear();
        edges.shrink_to_fit();
        auto deg = [&](int32_t c) { return aptr[c + 1] - aptr[c]; };
        for (int64_t c = 0; c < nc; ++c)
            std::sort(adj.begin() + aptr[c], adj.begin() + aptr[c + 1], [&](int32_t a, int32_t b) {
                return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
            });
        std::vector<int32_t> level(nc, -1), order;
        order.reserve(nc);
        // breadth-first levels from s over unvisited cells; returns the depth
        auto levels_from = [&](int32_t s, std::vector<int32_t>& out) -> int32_t {
            out.clear();
            out.push_back(s);
            level[s] = 0;
            for (size_t h = 0; h < out.size(); ++h) {
                const int32_t c = out[h];
                for (int64_t e = aptr[c]; e < aptr[c + 1]; ++e)
                    if (level[adj[e]] < 0) { level[adj[e]] = level[c] + 1; out.push_back(adj[e]); }
            }
            return level[out.back()];
        };
        std::vector<int32_t> by_mesh(nc);
        std::iota(by_mesh.begin(), by_mesh.end(), 0);
        std::stable_sort(by_mesh.begin(), by_mesh.end(),
                         [&](int32_t a, int32_t b) { return mesh_of_user[a] < mesh_of_user[b]; });
        std::vector<char> done(nc, 0);
        std::vector<int32_t> comp;
        for (size_t q = 0; q < by_mesh.size(); ++q) {
            const int32_t c0 = by_mesh[q];
            if (done[c0]) continue;
            // lowest-degree cell of this component as the first start
            int32_t s = c0;
            levels_from(c0, comp);
            for (int32_t c : comp) if (deg(c) < deg(s) || (deg(c) == deg(s) && c < s)) s = c;
            for (int32_t c : comp) level[c] = -1;
            int32_t depth = levels_from(s, comp);
            for (int it = 0; it < 8; ++it) {
                int32_t best = -1;
                for (int32_t c : comp)
                    if (level[c] == depth && (best < 0 || deg(c) < deg(best) || (deg(c) == deg(best) && c < best)))
                        best = c;
                for (int32_t c : comp) level[c] = -1;
                std::vector<int32_t> trial;
                const int32_t d2 = levels_from(best, trial);
                if (d2 <= depth) {
                    for (int32_t c : trial) level[c] = -1;
                    levels_from(s, comp);
                    break;
                }
                s = best;
                depth = d2;
                comp.swap(trial);
            }
            // comp is the breadth-first order from s (neighbours by degree)
            const size_t first = order.size();
            order.insert(order.end(), comp.begin(), comp.end());
            std::reverse(order.begin() + first, order.end());
            for (int32_t c : comp) done[c] = 1;
        }
        // components of a mesh stay in the order found; meshes in order
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return mesh_of_user[a] < mesh_of_user[b]; });
        if ((int64_t)order.size() != nc) { err = "internal error: renumbering lost cells"; return E_MESH; }
        new2old = order;
    } else if (renumber != 0) {
        err = "unknown renumbering";
        return E_ARG;
    }
    for (int64_t i = 0; i < nc; ++i) old2new[new2old[i]] = (int32_t)i;

    mark("renumbering");
    // -- 3. faces: sorted vertex triples, grouped (counting sort on a) -------
    static const int opp[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    std::vector<FaceRec> rec(4 * nc);
    std::vector<int64_t> bucket(nv + 1, 0);
    {
        std::vector<FaceRec> tmp(4 * nc);
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < 4; ++k) {
                int32_t v[3] = {T[c][opp[k][0]], T[c][opp[k][1]], T[c][opp[k][2]]};
                std::sort(v, v + 3);
                tmp[4 * c + k] = {v[0], v[1], v[2], (int32_t)c};
                bucket[v[0] + 1]++;
            }
        for (int64_t v = 0; v < nv; ++v) bucket[v + 1] += bucket[v];
        std::vector<int64_t> pos(bucket.begin(), bucket.end() - 1);
        for (auto& r : tmp) rec[pos[r.a]++] = r;
        for (int64_t v = 0; v < nv; ++v)
            std::sort(rec.begin() + bucket[v], rec.begin() + bucket[v + 1],
                      [](const FaceRec& x, const FaceRec& y) {
                          if (x.b != y.b) return x.b < y.b;
                          if (x.c != y.c) return x.c < y.c;
                          return x.owner < y.owner;
                      });
    }
    struct UFace {
        int32_t a, b, c;
        int32_t L, R;   // user cells; R = -1 on the boundary
        int32_t tag;
        int32_t bidx;   // index of the caller's boundary triangle (boundary faces)
    };
    std::vector<UFace> uf;
    uf.reserve(2 * nc + nb_in);
    for (size_t i = 0; i < rec.size();) {
        size_t j = i + 1;
        while (j < rec.size() && rec[j].a == rec[i].a && rec[j].b == rec[i].b && rec[j].c == rec[i].c) ++j;
        if (j - i > 2) { err = "face shared by more than two cells"; return E_MESH; }
        if (j - i == 2 && mesh_of_user[rec[i].owner] != mesh_of_user[rec[i + 1].owner]) {
            err = "a face is shared by cells of two different meshes";
            return E_MESH;
        }
        uf.push_back({rec[i].a, rec[i].b, rec[i].c, rec[i].owner, j - i == 2 ? rec[i + 1].owner : -1, -1, -1});
        i = j;
    }
    rec.clear();
    rec.shrink_to_fit();

    mark("faces");
    // -- 4. boundary tags ------------------------------------------------------
    auto less3 = [](const UFace& x, int32_t a, int32_t b, int32_t c) {
        if (x.a != a) return x.a < a;
        if (x.b != b) return x.b < b;
        return x.c < c;
    };
    for (int64_t i = 0; i < nb_in; ++i) {
        int32_t v[3] = {btris[3 * i], btris[3 * i + 1], btris[3 * i + 2]};
        std::sort(v, v + 3);
        auto it = std::lower_bound(uf.begin(), uf.end(), 0,
                                   [&](const UFace& x, int) { return less3(x, v[0], v[1], v[2]); });
        if (it == uf.end() || it->a != v[0] || it->b != v[1] || it->c != v[2] || it->R >= 0) {
            err = "tagged triangle is not a boundary face";
            return E_MESH;
        }
        if (it->tag >= 0) { err = "boundary face tagged twice"; return E_MESH; }
        it->tag = btags[i];
        it->bidx = (int32_t)i;
    }
    int64_t nb = 0, nfi = 0;
    for (auto& f : uf) {
        if (f.R < 0) {
            if (f.tag < 0) { err = "untagged boundary face"; return E_MESH; }
            ++nb;
        } else {
            ++nfi;
        }
    }
    const int64_t nf = nfi + nb;

    // -- 5. face orientation: S = 1/2 (B-A)x(C-A) points from L outwards ----
    for (auto& f : uf) {
        V3 A = P(f.a), B = P(f.b), C = P(f.c);
        V3 S = scale(cross(sub(B, A), sub(C, A)), 0.5);
        V3 xf = scale(add(add(A, B), C), 1.0 / 3.0);
        if (dot(S, sub(xf, cen_u[f.L])) < 0) std::swap(f.b, f.c);
    }

    mark("tags+orientation");
    // -- 6. internal face order ------------------------------------------------
    std::vector<int64_t> ford(uf.size());
    std::iota(ford.begin(), ford.end(), 0);
    auto fkey = [&](int64_t i) {
        const UFace& f = uf[i];
        int64_t l = old2new[f.L];
        if (f.R < 0) return std::array<int64_t, 3>{1, l, i};
        int64_t r = old2new[f.R];
        return std::array<int64_t, 3>{0, std::min(l, r) * (nc + 1) + std::max(l, r), i};
    };
    std::sort(ford.begin(), ford.end(), [&](int64_t x, int64_t y) { return fkey(x) < fkey(y); });

    mark("face order");
    // -- 7. vertex renumbering: by the first internal cell touching it ---------
    std::vector<int64_t> vmin(nv, INT64_MAX);
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < 4; ++k) vmin[T[c][k]] = std::min<int64_t>(vmin[T[c][k]], old2new[c]);
    for (int64_t v = 0; v < nv; ++v)
        if (vmin[v] == INT64_MAX) { err = "vertex not used by any cell"; return E_MESH; }
    std::vector<int32_t> vnew2old(nv), vold2new(nv);
    std::iota(vnew2old.begin(), vnew2old.end(), 0);
    std::stable_sort(vnew2old.begin(), vnew2old.end(), [&](int32_t a, int32_t b) { return vmin[a] < vmin[b]; });
    for (int64_t v = 0; v < nv; ++v) vold2new[vnew2old[v]] = (int32_t)v;

    // -- 8. fill internal arrays ------------------------------------------------
    M = Mesh();
    M.nc = nc; M.nv = nv; M.nf = nf; M.nfi = nfi; M.nb = nb;
    M.mesh_start = mstart;
    M.cell_perm = new2old;
    M.vert_perm = vnew2old;
    M.vol.resize(nc);
    M.xc.assign(3 * (nc + nb), 0.0);
    const int64_t NX = nc + nb;
    for (int64_t i = 0; i < nc; ++i) {
        int32_t o = new2old[i];
        M.vol[i] = vol_u[o];
        M.xc[i] = cen_u[o].x; M.xc[NX + i] = cen_u[o].y; M.xc[2 * NX + i] = cen_u[o].z;
    }
    M.fL.resize(nf); M.fR.resize(nf); M.fA.resize(nf); M.fB.resize(nf); M.fC.resize(nf);
    M.kAC.resize(nf); M.kBC.resize(nf); M.kRL.resize(nf); M.area.resize(nf);
    M.fx.resize(3 * nf); M.S.resize(3 * nf);
    M.gowner.resize(nb); M.gtag.resize(nb); M.gdist.resize(nb); M.gbtri.resize(nb);
    for (int64_t f = 0; f < nf; ++f) {
        const UFace& u = uf[ford[f]];
        V3 A = P(u.a), B = P(u.b), C = P(u.c);
        V3 S = scale(cross(sub(B, A), sub(C, A)), 0.5);
        V3 xf = scale(add(add(A, B), C), 1.0 / 3.0);
        int32_t L = old2new[u.L];
        V3 xL = cen_u[u.L];
        V3 xR;
        int32_t R;
        if (u.R >= 0) {
            R = old2new[u.R];
            xR = cen_u[u.R];
        } else {
            int64_t g = f - nfi;
            R = (int32_t)(nc + g);
            double a = std::sqrt(dot(S, S));
            V3 nh = scale(S, 1.0 / a);
            xR = add(xL, scale(nh, 2.0 * dot(sub(xf, xL), nh)));
            M.gowner[g] = L;
            M.gtag[g] = u.tag;
            M.gbtri[g] = u.bidx;
            V3 d = sub(xR, xL);
            M.gdist[g] = std::sqrt(dot(d, d));
            M.xc[nc + g] = xR.x; M.xc[NX + nc + g] = xR.y; M.xc[2 * NX + nc + g] = xR.z;
        }
        // diamond (eq. (diamond) with D = C): dual basis of {A-C, B-C, R-L}
        V3 cvec = sub(xR, xL);
        double muD = dot(S, cvec) / 3.0;
        if (!(muD > 0)) { err = "non-positive diamond volume"; return E_MESH; }
        V3 N1 = scale(cross(sub(B, C), cvec), 0.5);
        V3 N2 = scale(cross(cvec, sub(A, C)), 0.5);
        M.kAC[f] = dot(N1, S) / (3.0 * muD);
        M.kBC[f] = dot(N2, S) / (3.0 * muD);
        M.kRL[f] = dot(S, S) / (3.0 * muD);
        M.fL[f] = L; M.fR[f] = R;
        M.fA[f] = vold2new[u.a]; M.fB[f] = vold2new[u.b]; M.fC[f] = vold2new[u.c];
        M.fx[f] = xf.x; M.fx[nf + f] = xf.y; M.fx[2 * nf + f] = xf.z;
        M.S[f] = S.x; M.S[nf + f] = S.y; M.S[2 * nf + f] = S.z;
        M.area[f] = std::sqrt(dot(S, S));
    }
    uf.clear();
    uf.shrink_to_fit();

    mark("face geometry");
    // -- 9. cell -> faces ---------------------------------------------------------
    M.c2f.assign(4 * nc, -1);
    M.c2n.assign(4 * nc, -1);
    std::vector<int8_t> cnt(nc, 0);
    auto put = [&](int32_t cell, int32_t code, int32_t nbr) -> bool {
        if (cnt[cell] >= 4) return false;
        M.c2f[cnt[cell] * nc + cell] = code;
        M.c2n[cnt[cell] * nc + cell] = nbr;
        cnt[cell]++;
        return true;
    };
    for (int64_t f = 0; f < nf; ++f) {
        if (!put(M.fL[f], (int32_t)f, M.fR[f])) { err = "cell with more than 4 faces"; return E_MESH; }
        if (f < nfi && !put(M.fR[f], ~(int32_t)f, M.fL[f])) { err = "cell with more than 4 faces"; return E_MESH; }
    }
    for (int64_t c = 0; c < nc; ++c)
        if (cnt[c] != 4) { err = "cell without 4 faces"; return E_MESH; }

    mark("cell->face");
    // -- 10. vertex -> cells and ghosts ------------------------------------------
    {
        std::vector<int64_t> deg(nv + 1, 0);
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < 4; ++k) deg[vold2new[T[c][k]] + 1]++;
        for (int64_t g = 0; g < nb; ++g) {
            int64_t f = nfi + g;
            deg[M.fA[f] + 1]++; deg[M.fB[f] + 1]++; deg[M.fC[f] + 1]++;
        }
        for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
        M.nptr = deg;
        M.nidx.assign(M.nptr[nv], 0);
        std::vector<int64_t> pos(M.nptr.begin(), M.nptr.end() - 1);
        for (int64_t i = 0; i < nc; ++i) {   // internal order -> ascending per vertex
            const auto& t = T[new2old[i]];
            for (int k = 0; k < 4; ++k) M.nidx[pos[vold2new[t[k]]]++] = (int32_t)i;
        }
        for (int64_t g = 0; g < nb; ++g) {
            int64_t f = nfi + g;
            for (int32_t v : {M.fA[f], M.fB[f], M.fC[f]}) M.nidx[pos[v]++] = (int32_t)(nc + g);
        }
    }
    M.node_max = 0;
    M.n_len.assign(nv, 0);
    for (int64_t v = 0; v < nv; ++v) {
        M.n_len[v] = int32_t(M.nptr[v + 1] - M.nptr[v]);
        M.node_max = std::max<int32_t>(M.node_max, M.n_len[v]);
    }

    mark("vertex lists");
    // -- 11. least-squares vertex weights (Algorithm 2) -------------------------
    M.nalpha.assign(M.nidx.size(), 0.0);
    for (int64_t v = 0; v < nv; ++v) {
        V3 xv = P(vnew2old[v]);
        double A[4][4] = {{0}};
        for (int64_t e = M.nptr[v]; e < M.nptr[v + 1]; ++e) {
            int32_t id = M.nidx[e];
            double r[4] = {1.0, M.xc[id] - xv.x, M.xc[NX + id] - xv.y, M.xc[2 * NX + id] - xv.z};
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) A[i][j] += r[i] * r[j];
        }
        double rhs[4] = {1, 0, 0, 0}, w[4];
        if (!solve4(A, rhs, w)) { err = "singular vertex least-squares system"; return E_MESH; }
        for (int64_t e = M.nptr[v]; e < M.nptr[v + 1]; ++e) {
            int32_t id = M.nidx[e];
            M.nalpha[e] = w[0] + w[1] * (M.xc[id] - xv.x) + w[2] * (M.xc[NX + id] - xv.y) +
                          w[3] * (M.xc[2 * NX + id] - xv.z);
        }
    }

    mark("vertex weights");
    // -- 12. node-neighbour stencil (Algorithm 1): merge of 4 sorted lists ----
    M.sptr.assign(nc + 1, 0);
    M.sidx.clear();
    M.eptr.assign(nc + 1, 0);
    M.eidx.clear();
    M.eidx.reserve(size_t(nc) * 16);
    M.enbr_max = 0;
    M.sidx.reserve(size_t(nc) * 72);
    M.minv.assign(6 * nc, 0.0);
    M.klen.assign(nc, 0);
    M.stencil_max = 0;
    M.row_max = 0;
    for (int64_t i = 0; i < nc; ++i) {
        const auto& t = T[new2old[i]];
        int64_t h[4], e[4];
        for (int k = 0; k < 4; ++k) {
            int32_t v = vold2new[t[k]];
            h[k] = M.nptr[v];
            e[k] = M.nptr[v + 1];
        }
        int faces_seen = 0;
        int64_t last = -1;
        double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
        int32_t klen = 0;
        for (;;) {
            int64_t best = INT64_MAX;
            for (int k = 0; k < 4; ++k)
                if (h[k] < e[k]) best = std::min<int64_t>(best, M.nidx[h[k]]);
            if (best == INT64_MAX) break;
            int shared = 0;           // vertices of i whose list holds `best`
            for (int k = 0; k < 4; ++k)
                if (h[k] < e[k] && M.nidx[h[k]] == best) { ++h[k]; ++shared; }
            if (best == last || best == i) continue;
            last = best;
            if (shared == 2) {
                M.eidx.push_back((int32_t)best);
            } else if (shared == 3) {
                bool is_face = false;
                for (int k = 0; k < 4; ++k) is_face |= M.c2n[k * nc + i] == (int32_t)best;
                if (!is_face) { err = "entity sharing 3 vertices is not a face neighbour"; return E_MESH; }
                ++faces_seen;
            }
            M.sidx.push_back((int32_t)best);
            if (best < nc) ++klen;
            double dx = M.xc[best] - M.xc[i], dy = M.xc[NX + best] - M.xc[NX + i],
                   dz = M.xc[2 * NX + best] - M.xc[2 * NX + i];
            m00 += dx * dx; m01 += dx * dy; m02 += dx * dz;
            m11 += dy * dy; m12 += dy * dz; m22 += dz * dz;
        }
        if (faces_seen != 4) { err = "cell without 4 face-sharing stencil entities"; return E_MESH; }
        M.sptr[i + 1] = (int64_t)M.sidx.size();
        M.eptr[i + 1] = (int64_t)M.eidx.size();
        M.enbr_max = std::max<int32_t>(M.enbr_max, int32_t(M.eptr[i + 1] - M.eptr[i]));
        M.klen[i] = klen;
        M.stencil_max = std::max<int32_t>(M.stencil_max, int32_t(M.sptr[i + 1] - M.sptr[i]));
        M.row_max = std::max(M.row_max, klen);
        // inverse of the symmetric normal matrix by cofactors
        double c00 = m11 * m22 - m12 * m12, c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11;
        double c11 = m00 * m22 - m02 * m02, c12 = m01 * m02 - m00 * m12, c22 = m00 * m11 - m01 * m01;
        double det = m00 * c00 + m01 * c01 + m02 * c02;
        if (!(det > 0)) { err = "singular gradient normal matrix"; return E_MESH; }
        double id = 1.0 / det;
        M.minv[0 * nc + i] = c00 * id; M.minv[1 * nc + i] = c01 * id; M.minv[2 * nc + i] = c02 * id;
        M.minv[3 * nc + i] = c11 * id; M.minv[4 * nc + i] = c12 * id; M.minv[5 * nc + i] = c22 * id;
    }
    M.matrix_nnz = 0;
    for (int64_t i = 0; i < nc; ++i) M.matrix_nnz += M.klen[i] + 1;

    mark("stencil+gradient matrix");
    // -- 13. 64-row slicing ------------------------------------------------------
    pack_sell(M.sptr, M.sidx, nullptr, nullptr, nc, [](int64_t r) { return (int32_t)r; }, M.stencil);
    pack_sell(M.nptr, M.nidx, &M.nalpha, nullptr, nv,
              [&](int64_t r) { return M.nidx[M.nptr[r]]; }, M.node);
    if (!no_matrix)
        pack_sell(M.sptr, M.sidx, nullptr, &M.klen, nc, [](int64_t r) { return (int32_t)r; }, M.kmat);
    pack_sell(M.eptr, M.eidx, nullptr, nullptr, nc, [](int64_t r) { return (int32_t)r; }, M.enbr);

    mark("slicing");
    // -- 14. tiles and their halos -------------------------------------------------
    const int64_t kHaloCap = 2048;            // 64 KB of LDS at 32 bytes per entity
    std::vector<int64_t> seen(nc + nb, -1);      // last tile that collected the entity
    for (int32_t T = 256; T >= 64; T /= 2) {
        M.tile_rows = T;
        const int64_t nt = (nc + T - 1) / T;
        M.h_off.assign(nt + 1, 0);
        M.h_idx.clear();
        M.h_idx.reserve(size_t(nc) * 6);
        M.h_self.assign(nt, 0);
        M.halo_max = 0;
        std::fill(seen.begin(), seen.end(), -1);
        std::vector<int32_t> buf;
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t t0 = t * T, t1 = std::min(nc, t0 + T);
            buf.clear();
            for (int64_t i = t0; i < t1; ++i) {
                seen[i] = t;
                buf.push_back((int32_t)i);
            }
            for (int64_t e = M.sptr[t0]; e < M.sptr[t1]; ++e) {
                const int32_t v = M.sidx[e];
                if (seen[v] != t) {
                    seen[v] = t;
                    buf.push_back(v);
                }
            }
            std::sort(buf.begin(), buf.end());
            M.h_self[t] = int32_t(std::lower_bound(buf.begin(), buf.end(), (int32_t)t0) - buf.begin());
            M.h_idx.insert(M.h_idx.end(), buf.begin(), buf.end());
            M.h_off[t + 1] = (int64_t)M.h_idx.size();
            M.halo_max = std::max<int32_t>(M.halo_max, (int32_t)buf.size());
        }
        if (M.halo_max <= kHaloCap || T == 64) break;
    }
    if (M.halo_max > kHaloCap) { err = "stencil neighbourhood too large for the LDS tile"; return E_MESH; }
    mark("tile halos");
    // vertices of each tile (vertices are ordered by their lowest cell)
    {
        const int64_t nt = (int64_t)M.h_self.size();
        M.v_off.assign(nt + 1, 0);
        for (int64_t v = 0; v < nv; ++v) M.v_off[vmin[vnew2old[v]] / M.tile_rows + 1]++;
        for (int64_t t = 0; t < nt; ++t) M.v_off[t + 1] += M.v_off[t];
    }
    // global -> local through a dense map filled for one tile at a time
    M.n_lidx.assign(M.node.idx.size(), 0);
    M.k_lidx.assign(M.kmat.idx.size(), 0);
    M.c2n_l.assign(4 * nc, 0);
    M.e_lidx.assign(M.enbr.idx.size(), 0);
    M.c2v_l.assign(4 * nc, 0);
    std::vector<int64_t> fptr(1, 0);
    std::vector<int32_t> fent;                 // foreign lists, local halo indices
    M.fv_off.assign(M.h_self.size() + 1, 0);
    M.fv_idx.clear();
    M.fv_len.clear();
    M.tv_max = 0;
    const auto& cell_verts = T;
    {
        std::vector<int32_t> g2l(nc + nb, -1);
        std::vector<int32_t> v2l(nv, -1);
        const int64_t T = M.tile_rows;
        const int64_t nt = (int64_t)M.h_self.size();
        for (int64_t t = 0; t < nt; ++t) {
            for (int64_t h = M.h_off[t]; h < M.h_off[t + 1]; ++h) g2l[M.h_idx[h]] = int32_t(h - M.h_off[t]);
            const int64_t t0 = t * T, t1 = std::min(nc, t0 + T);
            for (int64_t r = t0; r < t1; ++r) {
                const int64_t sl = r >> 6;
                const int lane = int(r & 63);
                for (int64_t k = 0; !no_matrix && k < M.kmat.width[sl]; ++k) {
                    const int64_t at = M.kmat.off[sl] + k * 64 + lane;
                    M.k_lidx[at] = (uint16_t)g2l[M.kmat.idx[at]];
                }
                for (int k = 0; k < 4; ++k) M.c2n_l[k * nc + r] = (uint16_t)g2l[M.c2n[k * nc + r]];
                for (int64_t k = 0; k < M.enbr.width[sl]; ++k) {
                    const int64_t at = M.enbr.off[sl] + k * 64 + lane;
                    M.e_lidx[at] = (uint16_t)g2l[M.enbr.idx[at]];
                }
            }
            // vertices the tile's cells touch: own first, then foreign (sorted)
            const int64_t own = M.v_off[t + 1] - M.v_off[t];
            for (int64_t v = M.v_off[t]; v < M.v_off[t + 1]; ++v) v2l[v] = int32_t(v - M.v_off[t]);
            const size_t fbeg = M.fv_idx.size();
            for (int64_t r = t0; r < t1; ++r) {
                const auto& tt = cell_verts[new2old[r]];
                for (int k = 0; k < 4; ++k) {
                    const int32_t v = vold2new[tt[k]];
                    if (v2l[v] == -1) { v2l[v] = -2; M.fv_idx.push_back(v); }
                }
            }
            std::sort(M.fv_idx.begin() + fbeg, M.fv_idx.end());
            for (size_t q = fbeg; q < M.fv_idx.size(); ++q) {
                const int32_t v = M.fv_idx[q];
                v2l[v] = int32_t(own + int64_t(q - fbeg));
                M.fv_len.push_back(M.n_len[v]);
                for (int64_t e = M.nptr[v]; e < M.nptr[v + 1]; ++e) {
                    const int32_t l = g2l[M.nidx[e]];
                    if (l < 0) { err = "internal error: vertex list outside the tile halo"; return E_MESH; }
                    fent.push_back(l);
                }
                fptr.push_back((int64_t)fent.size());
            }
            M.fv_off[t + 1] = (int64_t)M.fv_idx.size();
            M.tv_max = std::max<int32_t>(M.tv_max, int32_t(own + int64_t(M.fv_idx.size() - fbeg)));
            for (int64_t r = t0; r < t1; ++r) {
                const auto& tt = cell_verts[new2old[r]];
                for (int k = 0; k < 4; ++k) M.c2v_l[k * nc + r] = (uint16_t)v2l[vold2new[tt[k]]];
            }
            for (int64_t v = M.v_off[t]; v < M.v_off[t + 1]; ++v) v2l[v] = -1;
            for (size_t q = fbeg; q < M.fv_idx.size(); ++q) v2l[M.fv_idx[q]] = -1;
            for (int64_t v = M.v_off[t]; v < M.v_off[t + 1]; ++v) {
                const int64_t sl = v >> 6;
                const int lane = int(v & 63);
                for (int64_t k = 0; k < M.node.width[sl]; ++k) {
                    const int64_t at = M.node.off[sl] + k * 64 + lane;
                    const int32_t l = g2l[M.node.idx[at]];
                    if (l < 0) { err = "internal error: vertex list outside its tile halo"; return E_MESH; }
                    M.n_lidx[at] = (uint16_t)l;
                }
            }
            for (int64_t h = M.h_off[t]; h < M.h_off[t + 1]; ++h) g2l[M.h_idx[h]] = -1;
        }
    }
    {   // foreign vertex lists in 64-row slices (pad = the row's first entry)
        const int64_t nfr = (int64_t)M.fv_idx.size();
        pack_sell(fptr, fent, nullptr, nullptr, nfr, [&](int64_t r) { return fent[fptr[r]]; }, M.fnode);
        M.f_lidx.assign(M.fnode.idx.begin(), M.fnode.idx.end());
        M.fnode.idx.clear();
        M.fnode.idx.shrink_to_fit();
    }
    mark("local indices");
    // every local index must name the same entity as the global one
    auto verify = [&](const Sell64& sl, const std::vector<uint16_t>& loc) -> bool {
        for (int64_t s_ = 0; s_ < sl.nslices; ++s_)
            for (int lane = 0; lane < 64; ++lane) {
                const int64_t r = s_ * 64 + lane;
                if (r >= nc) continue;
                const int64_t t = r / M.tile_rows;
                for (int64_t k = 0; k < sl.width[s_]; ++k) {
                    const int64_t at = sl.off[s_] + k * 64 + lane;
                    if (int64_t(loc[at]) >= M.h_off[t + 1] - M.h_off[t] || M.h_idx[M.h_off[t] + loc[at]] != sl.idx[at])
                        return false;
                }
            }
        return true;
    };
    bool ok = verify(M.kmat, M.k_lidx) && verify(M.enbr, M.e_lidx);
    for (int64_t i = 0; ok && i < nc; ++i) {
        const int64_t t = i / M.tile_rows;
        ok = M.h_idx[M.h_off[t] + M.h_self[t] + (i - t * M.tile_rows)] == i;
        for (int k = 0; ok && k < 4; ++k) ok = M.h_idx[M.h_off[t] + M.c2n_l[k * nc + i]] == M.c2n[k * nc + i];
    }
    if (!ok) { err = "internal error: tile-local index mismatch"; return E_MESH; }
    mark("verification");
    return 0;
}

}  // namespace mifvm
