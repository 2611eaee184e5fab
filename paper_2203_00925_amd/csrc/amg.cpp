// Host setup of the aggregation multigrid hierarchy (strength, aggregates,
// Galerkin coarse matrices, dense coarsest inverse).
#include "amg.h"

#include <algorithm>
#include <cmath>

#include "mifvm.h"

namespace mifvm {
namespace {

constexpr int E_ARG = MIFVM_E_ARG;

// strong neighbours of every row, in column order, with |a_ij|: counted,
// then written, row-parallel
void strength(const AmgCsr& A, double theta, std::vector<int64_t>& sptr, std::vector<int32_t>& sidx,
              std::vector<double>& sval) {
    sptr.assign(A.n + 1, 0);
    const int nt = setup_threads(A.n);
    auto row_max = [&](int64_t i) {
        double mx = 0.0;
        for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
            if (A.col[e] != i) mx = std::max(mx, std::fabs(A.val[e]));
        return mx;
    };
    auto strong = [&](int64_t i, int64_t e, double mx) {
        return mx > 0.0 && A.col[e] != i && std::fabs(A.val[e]) >= theta * mx;
    };
    for_chunks(A.n, nt, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const double mx = row_max(i);
            int64_t c = 0;
            for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) c += strong(i, e, mx) ? 1 : 0;
            sptr[i + 1] = c;
        }
    });
    for (int64_t i = 0; i < A.n; ++i) sptr[i + 1] += sptr[i];
    sidx.assign(sptr[A.n], 0);
    sval.assign(sptr[A.n], 0.0);
    for_chunks(A.n, nt, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const double mx = row_max(i);
            int64_t at = sptr[i];
            for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)
                if (strong(i, e, mx)) {
                    sidx[at] = A.col[e];
                    sval[at] = std::fabs(A.val[e]);
                    ++at;
                }
        }
    });
}

int64_t aggregate(const AmgCsr& A, const std::vector<int64_t>& sptr, const std::vector<int32_t>& sidx,
                  const std::vector<double>& sval, std::vector<int32_t>& agg) {
    const int64_t n = A.n;
    agg.assign(n, -1);
    int64_t na = 0;
    // pass 1: a row whose strong neighbours are all free seeds an aggregate
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        bool free = true;
        for (int64_t e = sptr[i]; e < sptr[i + 1] && free; ++e) free = agg[sidx[e]] < 0;
        if (!free) continue;
        agg[i] = int32_t(na);
        for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e) agg[sidx[e]] = int32_t(na);
        ++na;
    }
    // pass 2: join the aggregate of the strongest aggregated strong neighbour
    std::vector<int32_t> agg1 = agg;      // the aggregates of pass 1 only
    for (int64_t i = 0; i < n; ++i) {
        if (agg1[i] >= 0) continue;
        double best = -1.0;
        int32_t pick = -1;
        for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e) {
            const int32_t j = sidx[e];
            if (agg1[j] < 0) continue;
            const double w = sval[e];
            if (w > best || (w == best && j < pick)) {
                best = w;
                pick = j;
            }
        }
        if (pick >= 0) agg[i] = agg1[pick];
    }
    // pass 3: what is left seeds aggregates with its free strong neighbours
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        agg[i] = int32_t(na);
        for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e)
            if (agg[sidx[e]] < 0) agg[sidx[e]] = int32_t(na);
        ++na;
    }
    return na;
}

// A_c = P^T A P: coarse row I sums the rows of its members, columns mapped
// to aggregates; columns sorted
void galerkin(const AmgCsr& A, const std::vector<int32_t>& agg, int64_t na, AmgCsr& C) {
    std::vector<int64_t> mptr(na + 1, 0);
    for (int64_t i = 0; i < A.n; ++i) mptr[agg[i] + 1]++;
    for (int64_t a = 0; a < na; ++a) mptr[a + 1] += mptr[a];
    std::vector<int32_t> mem(A.n);
    {
        std::vector<int64_t> pos(mptr.begin(), mptr.end() - 1);
        for (int64_t i = 0; i < A.n; ++i) mem[pos[agg[i]]++] = int32_t(i);
    }
    C.n = na;
    C.ptr.assign(na + 1, 0);
    // coarse rows in contiguous chunks, one per thread, each into its own
    // buffers; then the chunks are concatenated in row order
    const int nt = setup_threads(A.n);
    std::vector<std::vector<int32_t>> pcol(nt);
    std::vector<std::vector<double>> pval(nt);
    for_chunks(na, nt, [&](int k, int64_t lo, int64_t hi) {
        std::vector<int32_t> slot(na, -1);
        std::vector<int32_t> cols, order;
        std::vector<double> acc;
        for (int64_t I = lo; I < hi; ++I) {
            cols.clear();
            acc.clear();
            for (int64_t m = mptr[I]; m < mptr[I + 1]; ++m) {
                const int64_t i = mem[m];
                for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
                    const int32_t J = agg[A.col[e]];
                    if (slot[J] < 0) {
                        slot[J] = int32_t(cols.size());
                        cols.push_back(J);
                        acc.push_back(0.0);
                    }
                    acc[slot[J]] += A.val[e];
                }
            }
            order.resize(cols.size());
            for (size_t q = 0; q < order.size(); ++q) order[q] = int32_t(q);
            std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cols[a] < cols[b]; });
            for (int32_t q : order) {
                pcol[k].push_back(cols[q]);
                pval[k].push_back(acc[q]);
            }
            for (int32_t J : cols) slot[J] = -1;
            C.ptr[I + 1] = int64_t(cols.size());
        }
    });
    for (int64_t I = 0; I < na; ++I) C.ptr[I + 1] += C.ptr[I];
    C.col.resize(C.ptr[na]);
    C.val.resize(C.ptr[na]);
    for_chunks(na, nt, [&](int k, int64_t lo, int64_t) {
        std::copy(pcol[k].begin(), pcol[k].end(), C.col.begin() + C.ptr[lo]);
        std::copy(pval[k].begin(), pval[k].end(), C.val.begin() + C.ptr[lo]);
    });
}

// dense inverse by LU with partial pivoting (row-major, n x n)
bool dense_inverse(const AmgCsr& A, std::vector<double>& inv) {
    const int64_t n = A.n;
    std::vector<double> M(n * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) M[i * n + A.col[e]] += A.val[e];
    std::vector<int64_t> piv(n);
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        for (int64_t r = k + 1; r < n; ++r)
            if (std::fabs(M[r * n + k]) > std::fabs(M[p * n + k])) p = r;
        if (!(std::fabs(M[p * n + k]) > 0.0)) return false;
        piv[k] = p;
        if (p != k)
            for (int64_t c = 0; c < n; ++c) std::swap(M[k * n + c], M[p * n + c]);
        const double d = M[k * n + k];
        for (int64_t r = k + 1; r < n; ++r) {
            const double l = M[r * n + k] / d;
            M[r * n + k] = l;
            if (l != 0.0)
                for (int64_t c = k + 1; c < n; ++c) M[r * n + c] -= l * M[k * n + c];
        }
    }
    inv.assign(n * n, 0.0);
    std::vector<double> x(n);
    for (int64_t c = 0; c < n; ++c) {           // column c of the inverse: solve A x = e_c
        std::fill(x.begin(), x.end(), 0.0);
        x[c] = 1.0;
        for (int64_t k = 0; k < n; ++k) std::swap(x[k], x[piv[k]]);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t k = 0; k < r; ++k) x[r] -= M[r * n + k] * x[k];
        for (int64_t r = n - 1; r >= 0; --r) {
            for (int64_t k = r + 1; k < n; ++k) x[r] -= M[r * n + k] * x[k];
            x[r] /= M[r * n + r];
        }
        for (int64_t r = 0; r < n; ++r) inv[r * n + c] = x[r];
    }
    return true;
}

}  // namespace

int amg_build(AmgCsr&& A, double theta, int max_levels, int64_t coarse_max, double omega, AmgHierarchy& H,
              std::string& err) {
    if (!(theta >= 0.0 && theta <= 1.0) || max_levels < 1 || max_levels > kAmgMaxLevels || coarse_max < 1 ||
        coarse_max > 4096 || !(omega > 0.0 && omega < 2.0)) {
        err = "bad multigrid options";
        return E_ARG;
    }
    if (A.n < 1) {
        err = "empty matrix";
        return E_ARG;
    }
    H = AmgHierarchy{};
    H.theta = theta;
    H.omega = omega;
    H.max_levels = max_levels;
    H.coarse_max = coarse_max;
    H.lv.emplace_back();
    H.lv[0].A = std::move(A);
    for (;;) {
        AmgLevel& L = H.lv.back();
        if (L.A.n <= coarse_max) break;
        if ((int)H.lv.size() == max_levels) {
            err = "coarsest level above coarse_max: raise max_levels";
            return E_ARG;
        }
        std::vector<int64_t> sptr;
        std::vector<int32_t> sidx;
        std::vector<double> sval;
        strength(L.A, theta, sptr, sidx, sval);
        const int64_t na = aggregate(L.A, sptr, sidx, sval, L.agg);
        if (na * 10 > L.A.n * 9) {
            err = "aggregation stalled (coarse level above 90% of the fine one)";
            return E_ARG;
        }
        L.ncoarse = na;
        AmgLevel next;
        galerkin(L.A, L.agg, na, next.A);
        H.lv.push_back(std::move(next));
    }
    if (!dense_inverse(H.lv.back().A, H.cinv)) {
        err = "singular coarsest matrix";
        return E_ARG;
    }
    return 0;
}

void amg_pack(const AmgCsr& A, Sell64& off, std::vector<double>& diag) {
    const int64_t n = A.n;
    diag.assign(n, 0.0);
    off.nslices = (n + 63) / 64;
    off.off.assign(off.nslices + 1, 0);
    off.width.assign(off.nslices, 0);
    std::vector<int32_t> len(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
            if (A.col[e] == i) diag[i] += A.val[e];
            else len[i]++;
        }
    for (int64_t s = 0; s < off.nslices; ++s) {
        int32_t w = 0;
        for (int64_t r = s * 64; r < std::min(n, s * 64 + 64); ++r) w = std::max(w, len[r]);
        off.width[s] = w;
        off.off[s + 1] = off.off[s] + int64_t(w) * 64;
    }
    off.idx.assign(off.off[off.nslices], 0);
    off.val.assign(off.off[off.nslices], 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s = i >> 6, lane = i & 63;
        int64_t k = 0;
        for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e) {
            if (A.col[e] == i) continue;
            off.idx[off.off[s] + k * 64 + lane] = A.col[e];
            off.val[off.off[s] + k * 64 + lane] = A.val[e];
            ++k;
        }
        for (; k < off.width[s]; ++k) off.idx[off.off[s] + k * 64 + lane] = int32_t(i);   // value 0
    }
}

}  // namespace mifvm
