// Kernels of the learned preconditioner (network forward, training backward,
// Adam) and of the flexible conjugate-gradient iteration that applies it.
//
// Work split of the network kernels: a wavefront takes 16 consecutive cells
// (a "group"); lane l works on cell l % 16 and owns row slots 8g..8g+7 of it,
// g = l / 16 (see nn_pi).  The per-cell products with W1 ([h; m] -> 32) and
// W2 (32 -> 32) are bf16 16x16x32 matrix-core operations with the weights as
// the A operand and the 16 cells' rows as the B operand, so each result tile
// leaves a lane exactly the features of its own slots.  A block (4 waves)
// walks 64-cell block-groups with a grid stride, the weights staying in
// registers.  Reductions over cells (loss, dot products, weight gradients)
// are per-block sums written with plain stores and added in block order by a
// separate kernel: deterministic for a fixed grid.
#include "nn.h"
#include "reduce.h"
#include "seg.h"
#include "state.h"

namespace mifvm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

constexpr int kFwdGridMax = 768;        // 3 blocks of 4 waves on each of 256 CUs (resident at once)

inline int nn_fwd_grid(int64_t nc) {
    const int64_t g = (nc + 63) / 64;
    return int(g < kFwdGridMax ? (g < 1 ? 1 : g) : kFwdGridMax);
}
inline int nn_bwd_grid(int64_t nc) {
    const int64_t g = (nc + 63) / 64;
    return int(g < kNnGridMax ? (g < 1 ? 1 : g) : kNnGridMax);
}

// bfloat16 <-> float (round to nearest even, as the oracle's rounding)
__device__ inline uint32_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float rbf(float f) { return __uint_as_float(f2bf(f) << 16); }

__device__ inline void unpack8(u32x4 v, float* o) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        o[2 * k] = __uint_as_float(v[k] << 16);
        o[2 * k + 1] = __uint_as_float(v[k] & 0xFFFF0000u);
    }
}
__device__ inline bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma16(i16x4 a, i16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// float pair -> packed bf16 pair (round to nearest even; one v_cvt_pk_bf16_f32)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t cvt2(float a, float b) {
    const f32x2 x = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2));
}
__device__ inline u32x4 cvt8(const float* f) {
    u32x4 v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = cvt2(f[2 * k], f[2 * k + 1]);
    return v;
}

// hi + lo split of FP32 values into two bf16 operands (about 16 mantissa bits)
__device__ inline void split8(const float* f, u32x4& hi, u32x4& lo) {
    hi = cvt8(f);
    float h[8], l[8];
    unpack8(hi, h);
#pragma unroll
    for (int j = 0; j < 8; ++j) l[j] = f[j] - h[j];
    lo = cvt8(l);
}

// Contiguous range of 64-cell block-groups of this block: consecutive cells
// stay on one XCD, whose L2 then serves the neighbour rows they share.
__device__ inline void block_range(int64_t nbg, int64_t& b0, int64_t& b1) {
    const int64_t per = (nbg + gridDim.x - 1) / gridDim.x;
    b0 = int64_t(blockIdx.x) * per;
    if (b0 > nbg) b0 = nbg;
    b1 = b0 + per < nbg ? b0 + per : nbg;
}

// tile of this block: blocks are dealt to the 8 XCDs in turn, so with the
// grid padded to a multiple of 8 each XCD takes a contiguous eighth of the
// tiles (neighbouring tiles share the cells of their rings in one L2)
__device__ inline int64_t xcd_tile(int64_t ntiles) {
    const int64_t per = gridDim.x / 8;
    return int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
}

struct NnIn {
    int64_t nc;
    const int4* nbr;
    const double* r64;        // input residual (one of r64 / r32)
    const float* r32;
    const double* dinv;
    const double* scal;       // mesh-0 scalar slots
    const NnPack* pack;
};

// h0 = We x + be of one cell (slots 8g..8g+7), rounded and packed
__device__ inline u32x4 encode(double r, double dv, const float* we0, const float* we1, const float* be,
                               double isr, double isd) {
    const float x0 = float(r * isr), x1 = float(dv * r * isd);
    float h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = fmaf(we0[j], x0, fmaf(we1[j], x1, be[j]));
    return cvt8(h);
}

// v = W1 [h; m] with m = 1/4 sum of the neighbour rows: the neighbour rows
// are further K-chunks of the product against W1's m-half scaled by 1/4
// (w1[t][1]), so m is summed in the FP32 accumulator and never rounded.
// Absent neighbours are zero rows.  Forward and backward use this one
// sequence, so the recomputed v is bitwise the forward's.
__device__ inline void w1_product(const bf16x8 (&w1)[2][2], u32x4 bh, const u32x4 (&bn)[4], f32x4 (&v)[2]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        v[t] = mfma32(w1[t][0], as_bf(bh), f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int k = 0; k < 4; ++k) v[t] = mfma32(w1[t][1], as_bf(bn[k]), v[t]);
    }
}

// ---- forward -------------------------------------------------------------------
// KIND 0: first layer (input encoded from r), 1: middle, 2: last (decoder and
// z = D^-1 r + s_d y).  FCG: return at once when the solve has finished, and
// write per-block partial sums of z.r and z.r_old.  KEEP: the last layer also
// stores its h (training).
//
// A block takes a contiguous range of 64-cell block-groups (so the neighbour
// rows its cells share are fetched into its XCD's L2 once); each of its waves
// walks every fourth 16-cell group of the range as a two-stage pipeline:
// while group k is computed, the rows of group k+1 (whose neighbour indices
// arrived during step k-1) and the neighbour indices of group k+2 are in
// flight, so the gather's two dependent loads overlap the matrix-core work.
struct NnFwd {
    NnIn in;
    const u32x4* hin;
    u32x4* hout;
    double* z;
    const double* r_old;
    double* partial;          // [2][gridDim.x]
    int layer;
};

// inputs of one group as loaded (rows or residual values of the cell and its
// face neighbours; absent ones are 0 and flagged by nb < 0)
template <int KIND>
struct FwdRaw {
    u32x4 h[5];               // KIND 1, 2: own row chunk, then the neighbours'
    double r[5], dv[5];       // KIND 0: r and D^-1 of the cell and neighbours
    double rs, ds, ro;        // KIND 2: own r, D^-1, r_old
};

__device__ inline int4 load_nbr(const NnIn& A, int64_t G, int64_t Gend, int c) {
    const int64_t i = G * 16 + c;
    return (G < Gend && i < A.nc) ? A.nbr[i] : make_int4(-1, -1, -1, -1);
}

template <int KIND, bool R32, bool FCG>
__device__ inline void load_raw(const NnFwd& F, int64_t G, int64_t Gend, int4 nb, int c, int g, FwdRaw<KIND>& w) {
    const NnIn& A = F.in;
    const int64_t i = G * 16 + c;
    const bool valid = G < Gend && i < A.nc;
    const int nbs[4] = {nb.x, nb.y, nb.z, nb.w};
    if (KIND == 0) {
        w.r[0] = valid ? (R32 ? double(A.r32[i]) : A.r64[i]) : 0.0;
        w.dv[0] = valid ? A.dinv[i] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            w.r[k + 1] = nbs[k] >= 0 ? (R32 ? double(A.r32[nbs[k]]) : A.r64[nbs[k]]) : 0.0;
            w.dv[k + 1] = nbs[k] >= 0 ? A.dinv[nbs[k]] : 0.0;
        }
    } else {
        const u32x4 z4 = {0u, 0u, 0u, 0u};
        w.h[0] = valid ? F.hin[i * 4 + g] : z4;
#pragma unroll
        for (int k = 0; k < 4; ++k) w.h[k + 1] = nbs[k] >= 0 ? F.hin[int64_t(nbs[k]) * 4 + g] : z4;
    }
    if (KIND == 2) {
        w.rs = valid ? (R32 ? double(A.r32[i]) : A.r64[i]) : 0.0;
        w.ds = valid ? A.dinv[i] : 0.0;
        w.ro = (FCG && valid) ? F.r_old[i] : 0.0;
    }
}

template <int KIND, bool R32, bool FCG, bool KEEP>
__global__ __launch_bounds__(256) void k_nn_layer(NnFwd F) {
    const NnIn& A = F.in;
    if (FCG && A.scal[SC_DONE] != 0.0) return;
    __shared__ double lds[4];
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const NnPack* P = A.pack;
    const NnPackLayer& L = P->layer[F.layer];
    bf16x8 w1[2][2], w2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        w1[t][0] = L.w1[t][0][lane];
        w1[t][1] = L.w1[t][1][lane];
        w2[t] = L.w2[t][lane];
    }
    float b1[8], b2[8], we0[8], we1[8], be[8], wd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        b1[j] = L.b1[8 * g + j];
        b2[j] = L.b2[8 * g + j];
        we0[j] = P->we0[8 * g + j];
        we1[j] = P->we1[8 * g + j];
        be[j] = P->be[8 * g + j];
        wd[j] = P->wd[8 * g + j];
    }
    const float bd = P->bd;
    const double isr = A.scal[SC_NN_INV_SR], isd = A.scal[SC_NN_INV_SD], sd = A.scal[SC_NN_SD];
    double zr = 0.0, zro = 0.0;
    int64_t b0, b1r;
    block_range((A.nc + 63) / 64, b0, b1r);
    const int64_t Gend = b1r * 4;
    int64_t G = b0 * 4 + wv;
    int4 nb_a = load_nbr(A, G, Gend, c);
    int4 nb_b = load_nbr(A, G + 4, Gend, c);
    FwdRaw<KIND> ra;
    load_raw<KIND, R32, FCG>(F, G, Gend, nb_a, c, g, ra);
    for (; G < Gend; G += 4) {
        FwdRaw<KIND> rb;
        load_raw<KIND, R32, FCG>(F, G + 4, Gend, nb_b, c, g, rb);
        const int4 nb_c = load_nbr(A, G + 8, Gend, c);
        const int64_t i = G * 16 + c;
        const bool valid = i < A.nc;
        const u32x4 z4 = {0u, 0u, 0u, 0u};
        u32x4 bh, bn[4];
        if (KIND == 0) {
            const int nbs[4] = {nb_a.x, nb_a.y, nb_a.z, nb_a.w};
            bh = valid ? encode(ra.r[0], ra.dv[0], we0, we1, be, isr, isd) : z4;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                bn[k] = nbs[k] >= 0 ? encode(ra.r[k + 1], ra.dv[k + 1], we0, we1, be, isr, isd) : z4;
        } else {
            bh = ra.h[0];
#pragma unroll
            for (int k = 0; k < 4; ++k) bn[k] = ra.h[k + 1];
        }
        float hown[8];
        unpack8(bh, hown);
        f32x4 v[2];
        w1_product(w1, bh, bn, v);
        float u[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) u[j] = fmaxf(v[j >> 2][j & 3] + b1[j], 0.f);
        const u32x4 bu = cvt8(u);
        float hf[8];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const f32x4 o = mfma32(w2[t], as_bf(bu), f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int k = 0; k < 4; ++k) hf[4 * t + k] = (hown[4 * t + k] + o[k]) + b2[4 * t + k];
        }
        const u32x4 hp = cvt8(hf);
        if ((KIND != 2 || KEEP) && valid) F.hout[i * 4 + g] = hp;
        if (KIND == 2) {
            float hn[8];
            unpack8(hp, hn);
            float y = 0.f;
#pragma unroll
            for (int j = 0; j < 8; ++j) y = fmaf(wd[j], hn[j], y);
            y += __shfl_xor(y, 16, 64);
            y += __shfl_xor(y, 32, 64);
            y += bd;
            if (g == 0 && valid) {
                const double zi = __fma_rn(sd, double(y), ra.ds * ra.rs);   // one rounding order in every forward
                F.z[i] = zi;
                if (FCG) {
                    zr += zi * ra.rs;
                    zro += zi * ra.ro;
                }
            }
        }
        nb_a = nb_b;
        nb_b = nb_c;
        ra = rb;
    }
    if (FCG && KIND == 2) {
        const double s0 = block_sum256(zr, lds);
        const double s1 = block_sum256(zro, lds);
        if (threadIdx.x == 0) {
            F.partial[blockIdx.x] = s0;
            F.partial[gridDim.x + blockIdx.x] = s1;
        }
    }
}

// ---- fused forward ----------------------------------------------------------------
// The three layers of one tile in one workgroup: the encoding of the tile's
// whole list (rings 0-3) goes to LDS as bf16 rows; layer 1 is evaluated on
// rings 0-2, layer 2 on rings 0-1, layer 3 and the decoder on ring 0 (the
// tile's own cells).  The first two layers keep their outputs in registers
// (at most kNnFusedMaxGroups 16-cell groups per wave, statically indexed)
// until every wave has read its inputs, then overwrite the rows in place; the
// last layer feeds the decoder directly.  A cell's arithmetic is the
// three-launch forward's (the same encode, products, roundings and decoder),
// so z is bitwise the same; only the rows of neighbouring cells are
// recomputed per tile instead of read from HBM.
//
// LDS rows are planar, [slot group g][list entry]: the 16 lanes of one slot
// group read 16 consecutive 16-byte rows of their own cells, which fall in
// distinct banks (the neighbour rows are random reads either way).
struct NnFused {
    NnIn in;
    const int64_t* ext_off;
    const int4* ring;
    const int32_t* cell;
    const int64_t* nb_off;
    const ushort4* nb;
    int64_t ntiles;
    int32_t ext_max;
    double* z;
    const double* r_old;
    double* partial;          // [2][ntiles]
};

// one network layer on the first N entries of the tile's list; LAST: the
// decoder and z of the tile's own cells (and the FCG dot partials).  Groups
// go in pairs of straight-line code, so the LDS reads and matrix-core chain
// of one group overlap the other's (a pair past N reads zero rows).
template <bool FCG, int L>
__device__ inline void fused_layer(const NnFused& F, u32x4* rows, int cap, const ushort4* lnb, int N, int lane,
                                   int wv, int64_t eo, double sd, double& zr, double& zro) {
    constexpr bool LAST = L == kNnLayers - 1;
    const int c = lane & 15, g = lane >> 4;
    const NnPack* P = F.in.pack;
    const NnPackLayer& Ly = P->layer[L];
    const u32x4* plane = rows + size_t(g) * cap;
    bf16x8 w1[2][2], w2[2];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        w1[tt][0] = Ly.w1[tt][0][lane];
        w1[tt][1] = Ly.w1[tt][1][lane];
        w2[tt] = Ly.w2[tt][lane];
    }
    float b1[8], b2[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        b1[j] = Ly.b1[8 * g + j];
        b2[j] = Ly.b2[8 * g + j];
    }
    const u32x4 z4 = {0u, 0u, 0u, 0u};
    // one 16-cell group: the layer's output slots of this lane
    auto group = [&](int G) -> u32x4 {
        const int e = G * 16 + c;
        const bool valid = e < N;
        const u32x4 bh = valid ? plane[e] : z4;
        const ushort4 nb = valid ? lnb[e] : make_ushort4(0xFFFF, 0xFFFF, 0xFFFF, 0xFFFF);
        const uint16_t nbs[4] = {nb.x, nb.y, nb.z, nb.w};
        u32x4 bn[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bn[q] = nbs[q] != 0xFFFF ? plane[nbs[q]] : z4;
        float hown[8];
        unpack8(bh, hown);
        f32x4 v[2];
        w1_product(w1, bh, bn, v);
        float u[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) u[j] = fmaxf(v[j >> 2][j & 3] + b1[j], 0.f);
        const u32x4 bu = cvt8(u);
        float hf[8];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const f32x4 o = mfma32(w2[tt], as_bf(bu), f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int q = 0; q < 4; ++q) hf[4 * tt + q] = (hown[4 * tt + q] + o[q]) + b2[4 * tt + q];
        }
        return cvt8(hf);
    };
    constexpr int W = kNnFusedWaves;
    if constexpr (LAST) {
        float wd[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) wd[j] = P->wd[8 * g + j];
        const float bd = P->bd;
        auto decode = [&](int G, u32x4 out) {
            float hn[8];
            unpack8(out, hn);
            float y = 0.f;
#pragma unroll
            for (int j = 0; j < 8; ++j) y = fmaf(wd[j], hn[j], y);
            y += __shfl_xor(y, 16, 64);
            y += __shfl_xor(y, 32, 64);
            y += bd;
            const int e = G * 16 + c;
            if (g == 0 && e < N) {
                const int64_t i = int64_t(F.cell[eo + e]);
                const double rs = F.in.r64[i], ds = F.in.dinv[i];
                const double zi = __fma_rn(sd, double(y), ds * rs);
                F.z[i] = zi;
                if (FCG) {
                    zr += zi * rs;
                    zro += zi * F.r_old[i];
                }
            }
        };
        for (int G = wv; G * 16 < N; G += 2 * W) {
            const u32x4 o0 = group(G);
            const u32x4 o1 = group(G + W);
            decode(G, o0);
            decode(G + W, o1);
        }
    } else {
        u32x4 out[kNnFusedMaxGroups];
#pragma unroll
        for (int k = 0; k < kNnFusedMaxGroups; k += 2) {
            const int G = wv + W * k;
            if (G * 16 < N) {                         // uniform over the wave
                out[k] = group(G);
                out[k + 1] = group(G + W);
            } else {
                out[k] = z4;
                out[k + 1] = z4;
            }
        }
        __syncthreads();                              // every wave has read the layer's inputs
        u32x4* wplane = rows + size_t(g) * cap;
#pragma unroll
        for (int k = 0; k < kNnFusedMaxGroups; ++k) {
            const int e = (wv + W * k) * 16 + c;
            if (e < N) wplane[e] = out[k];
        }
        __syncthreads();
    }
}

template <bool FCG>
__global__ __launch_bounds__(256) void k_nn_fused(NnFused F) {
    extern __shared__ __align__(16) unsigned char nn_smem[];
    const int cap = F.ext_max;
    u32x4* rows = reinterpret_cast<u32x4*>(nn_smem);                                  // [4][cap]
    ushort4* lnb = reinterpret_cast<ushort4*>(nn_smem + size_t(cap) * 64);            // [rings 0-2]
    __shared__ double lds[4];
    const NnIn& A = F.in;
    if (FCG && A.scal[SC_DONE] != 0.0) return;
    const int64_t t = xcd_tile(F.ntiles);
    if (t >= F.ntiles) return;
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const NnPack* P = A.pack;
    const int4 rn = F.ring[t];                       // cumulative ring sizes
    const int64_t eo = F.ext_off[t], no = F.nb_off[t];
    {   // one thread per list entry: every index and residual load goes out
        // at once; (r, D^-1 r) wait in plane 0 of the entry's row
        int cl[kNnFusedEntriesPerThread];
        ushort4 nbv[kNnFusedEntriesPerThread];
#pragma unroll
        for (int j = 0; j < kNnFusedEntriesPerThread; ++j) {
            const int e = threadIdx.x + 256 * j;
            cl[j] = F.cell[eo + (e < rn.w ? e : 0)];
            nbv[j] = F.nb[no + (e < rn.z ? e : 0)];
        }
        double rv[kNnFusedEntriesPerThread], dv[kNnFusedEntriesPerThread];
#pragma unroll
        for (int j = 0; j < kNnFusedEntriesPerThread; ++j) {
            rv[j] = A.r64[cl[j]];
            dv[j] = A.dinv[cl[j]];
        }
#pragma unroll
        for (int j = 0; j < kNnFusedEntriesPerThread; ++j) {
            const int e = threadIdx.x + 256 * j;
            if (e < rn.z) lnb[e] = nbv[j];
            if (e < rn.w) {
                u32x4 pk;
                const uint64_t rb = __double_as_longlong(rv[j]), db = __double_as_longlong(dv[j]);
                pk[0] = uint32_t(rb);
                pk[1] = uint32_t(rb >> 32);
                pk[2] = uint32_t(db);
                pk[3] = uint32_t(db >> 32);
                rows[e] = pk;
            }
        }
    }
    __syncthreads();
    {   // encoding of every cell of the list: the four lanes of a cell read
        // (r, D^-1) from plane 0 before the wave overwrites it
        float we0[8], we1[8], be[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            we0[j] = P->we0[8 * g + j];
            we1[j] = P->we1[8 * g + j];
            be[j] = P->be[8 * g + j];
        }
        const double isr = A.scal[SC_NN_INV_SR], isd = A.scal[SC_NN_INV_SD];
        u32x4* plane = rows + size_t(g) * cap;
        for (int G = wv; G * 16 < rn.w; G += kNnFusedWaves) {
            const int e = G * 16 + c;
            if (e < rn.w) {
                const u32x4 pk = rows[e];
                const double r = __longlong_as_double(int64_t(uint64_t(pk[0]) | (uint64_t(pk[1]) << 32)));
                const double d = __longlong_as_double(int64_t(uint64_t(pk[2]) | (uint64_t(pk[3]) << 32)));
                const u32x4 h = encode(r, d, we0, we1, be, isr, isd);
                __builtin_amdgcn_wave_barrier();
                plane[e] = h;
            }
        }
    }
    __syncthreads();
    const double sd = A.scal[SC_NN_SD];
    double zr = 0.0, zro = 0.0;
    static_assert(kNnLayers == 3, "the fused forward is written for three layers");
    fused_layer<FCG, 0>(F, rows, cap, lnb, rn.z, lane, wv, eo, sd, zr, zro);
    fused_layer<FCG, 1>(F, rows, cap, lnb, rn.y, lane, wv, eo, sd, zr, zro);
    fused_layer<FCG, 2>(F, rows, cap, lnb, rn.x, lane, wv, eo, sd, zr, zro);
    if (FCG) {
        const double s0 = block_sum256(zr, lds);
        const double s1 = block_sum256(zro, lds);
        if (threadIdx.x == 0) {
            F.partial[t] = s0;
            F.partial[F.ntiles + t] = s1;
        }
    }
}

// ---- backward ------------------------------------------------------------------
// Layer `layer` in reverse.  Input of the layer: h (TOP..: saved rows; FIRST:
// re-encoded from r).  Gradient reaching the layer's output:
//   TOP:  dh = dy wd with dy = s_d dz, dz = -2 w / ||r||^2, w = K^T (r - K z)
//   else: dh = base + 1/4 sum_{face neighbours j} dam_j   (from the layer above)
// The layer recomputes v = W1 [h; m] + b1 and u, then
//   du = (W2^T dh) * [v > 0],  da = W1^T du = [da_h; da_m],
//   base_out = dh + da_h,  dam_out = da_m,
// and adds dW2 = dh u^T, db2 = dh, dW1 = du [h; m]^T, db1 = du (TOP also dwd =
// dy h_out, dbd = dy) into per-block sums.  The data-path products split dh
// and du into bf16 hi + lo operands; the weight-gradient products transpose
// dh, du, u and [h; m] through LDS and run 16x16x16 bf16 tiles with the 16
// cells as the contraction.
struct NnBwd {
    NnIn in;
    const u32x4* hin;         // layer input rows (unused when FIRST)
    const u32x4* hout;        // TOP: rows of the last layer's output
    const double* w;          // TOP: K^T (r - K z)
    const float* base_in;     // !TOP
    const float* dam_in;
    float* base_out;
    float* dam_out;
    float* partial;           // [gridDim.x][kNnParams]
    int layer;
};

struct WaveT {                // per-wave transposes, [feature][cell] bf16
    uint16_t dh_hi[32][16], dh_lo[32][16], du_hi[32][16], du_lo[32][16], u[32][16], a[64][16];
    uint16_t m_lo[32][16];    // low part of the (unrounded) neighbour mean
};

__device__ inline i16x4 ld4(const uint16_t* p) { return *reinterpret_cast<const i16x4*>(p); }

template <bool FIRST, bool TOP>
__global__ __launch_bounds__(256) void k_nn_bwd(NnBwd B) {
    const NnIn& A = B.in;
    __shared__ __align__(16) WaveT wt[4];
    __shared__ float red[kNnLayerSize + 33];
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const NnPack* P = A.pack;
    const NnPackLayer& L = P->layer[B.layer];
    bf16x8 w1[2][2], w2t[2], w1t[4];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        w1[t][0] = L.w1[t][0][lane];
        w1[t][1] = L.w1[t][1][lane];
        w2t[t] = L.w2t[t][lane];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) w1t[t] = L.w1t[t][lane];
    float b1[8], we0[8], we1[8], be[8], wd[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        b1[j] = L.b1[8 * g + j];
        we0[j] = P->we0[8 * g + j];
        we1[j] = P->we1[8 * g + j];
        be[j] = P->be[8 * g + j];
        wd[j] = P->wd[8 * g + j];
    }
    const double isr = A.scal[SC_NN_INV_SR], isd = A.scal[SC_NN_INV_SD];
    const double dscale = A.scal[SC_NN_DSCALE];                 // dy = dscale * w (set by the loss)
    f32x4 gw2[2][2], gw1[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        gw2[a][0] = gw2[a][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gw1[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[8], gb2[8], gwd[8], gbd = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) gb1[j] = gb2[j] = gwd[j] = 0.f;
    WaveT& T = wt[wv];
    int64_t bg0, bg1;
    block_range((A.nc + 63) / 64, bg0, bg1);
    for (int64_t bg = bg0; bg < bg1; ++bg) {         // the same trip count in every wave
        const int64_t i = bg * 64 + wv * 16 + c;
        const bool valid = i < A.nc;
        const int4 nb = valid ? A.nbr[i] : make_int4(-1, -1, -1, -1);
        const int nbv[4] = {nb.x, nb.y, nb.z, nb.w};
        const u32x4 z4 = {0u, 0u, 0u, 0u};
        u32x4 bh, bn[4];
        if (FIRST) {
            bh = valid ? encode(double(A.r32[i]), A.dinv[i], we0, we1, be, isr, isd) : z4;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                bn[k] = nbv[k] >= 0 ? encode(double(A.r32[nbv[k]]), A.dinv[nbv[k]], we0, we1, be, isr, isd) : z4;
        } else {
            bh = valid ? B.hin[i * 4 + g] : z4;
#pragma unroll
            for (int k = 0; k < 4; ++k) bn[k] = nbv[k] >= 0 ? B.hin[int64_t(nbv[k]) * 4 + g] : z4;
        }
        float hown[8], m[8];
        unpack8(bh, hown);
#pragma unroll
        for (int j = 0; j < 8; ++j) m[j] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t[8];
            unpack8(bn[k], t);
#pragma unroll
            for (int j = 0; j < 8; ++j) m[j] += t[j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) m[j] *= 0.25f;
        f32x4 vv4[2];
        w1_product(w1, bh, bn, vv4);
        float u[8];
        bool on[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float vv = vv4[j >> 2][j & 3] + b1[j];
            on[j] = vv > 0.f;
            u[j] = fmaxf(vv, 0.f);
        }
        const u32x4 bu = cvt8(u);
        // gradient at the layer output
        float dh[8];
        if (TOP) {
            const float dy = valid ? float(dscale * B.w[i]) : 0.f;
            float ho[8];
            u32x4 z4 = {0u, 0u, 0u, 0u};
            unpack8(valid ? B.hout[i * 4 + g] : z4, ho);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                dh[j] = dy * wd[j];
                gwd[j] = fmaf(dy, ho[j], gwd[j]);
            }
            if (g == 0) gbd += dy;
        } else {
            const int nbs[4] = {nb.x, nb.y, nb.z, nb.w};
            float acc[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (nbs[k] < 0) continue;
                const float4* q = reinterpret_cast<const float4*>(B.dam_in + int64_t(nbs[k]) * 32 + 8 * g);
                const float4 q0 = q[0], q1 = q[1];
                acc[0] += q0.x; acc[1] += q0.y; acc[2] += q0.z; acc[3] += q0.w;
                acc[4] += q1.x; acc[5] += q1.y; acc[6] += q1.z; acc[7] += q1.w;
            }
            if (valid) {
                const float4* q = reinterpret_cast<const float4*>(B.base_in + i * 32 + 8 * g);
                const float4 q0 = q[0], q1 = q[1];
                const float bs[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                for (int j = 0; j < 8; ++j) dh[j] = bs[j] + 0.25f * acc[j];
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) dh[j] = 0.f;
            }
        }
        // du = (W2^T dh) * [v > 0]
        u32x4 dh_hi, dh_lo;
        split8(dh, dh_hi, dh_lo);
        float du[8];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x4 o = mfma32(w2t[t], as_bf(dh_hi), f32x4{0.f, 0.f, 0.f, 0.f});
            o = mfma32(w2t[t], as_bf(dh_lo), o);
#pragma unroll
            for (int k = 0; k < 4; ++k) du[4 * t + k] = on[4 * t + k] ? o[k] : 0.f;
        }
        // da = W1^T du
        u32x4 du_hi, du_lo;
        split8(du, du_hi, du_lo);
        float da_h[8], da_m[8];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 o = mfma32(w1t[t], as_bf(du_hi), f32x4{0.f, 0.f, 0.f, 0.f});
            o = mfma32(w1t[t], as_bf(du_lo), o);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (t < 2) da_h[4 * t + k] = o[k];
                else da_m[4 * (t - 2) + k] = o[k];
            }
        }
        if (valid) {
            float4* bo = reinterpret_cast<float4*>(B.base_out + i * 32 + 8 * g);
            float4* mo = reinterpret_cast<float4*>(B.dam_out + i * 32 + 8 * g);
            bo[0] = make_float4(dh[0] + da_h[0], dh[1] + da_h[1], dh[2] + da_h[2], dh[3] + da_h[3]);
            bo[1] = make_float4(dh[4] + da_h[4], dh[5] + da_h[5], dh[6] + da_h[6], dh[7] + da_h[7]);
            mo[0] = make_float4(da_m[0], da_m[1], da_m[2], da_m[3]);
            mo[1] = make_float4(da_m[4], da_m[5], da_m[6], da_m[7]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            gb2[j] += dh[j];
            gb1[j] += du[j];
        }
        // transposes for the weight gradients (invalid cells carry zero dh, du)
        {
            u32x4 m_hi, m_lo;
            split8(m, m_hi, m_lo);
            const u32x4 hh = dh_hi, hl = dh_lo, uh = du_hi, ulo = du_lo;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int f = nn_pi(8 * g + j);
                const int k = j >> 1, sh = (j & 1) * 16;
                T.dh_hi[f][c] = uint16_t(hh[k] >> sh);
                T.dh_lo[f][c] = uint16_t(hl[k] >> sh);
                T.du_hi[f][c] = uint16_t(uh[k] >> sh);
                T.du_lo[f][c] = uint16_t(ulo[k] >> sh);
                T.u[f][c] = uint16_t(bu[k] >> sh);
                T.a[f][c] = uint16_t(bh[k] >> sh);
                T.a[32 + f][c] = uint16_t(m_hi[k] >> sh);
                T.m_lo[f][c] = uint16_t(m_lo[k] >> sh);
            }
        }
        __syncthreads();
#pragma unroll
        for (int to = 0; to < 2; ++to) {
            const i16x4 ah = ld4(&T.dh_hi[16 * to + c][4 * g]), al = ld4(&T.dh_lo[16 * to + c][4 * g]);
            const i16x4 ch = ld4(&T.du_hi[16 * to + c][4 * g]), cl = ld4(&T.du_lo[16 * to + c][4 * g]);
#pragma unroll
            for (int ti = 0; ti < 2; ++ti) {
                const i16x4 bu = ld4(&T.u[16 * ti + c][4 * g]);
                gw2[to][ti] = mfma16(ah, bu, gw2[to][ti]);
                gw2[to][ti] = mfma16(al, bu, gw2[to][ti]);
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti) {
                const i16x4 ba = ld4(&T.a[16 * ti + c][4 * g]);
                gw1[to][ti] = mfma16(ch, ba, gw1[to][ti]);
                gw1[to][ti] = mfma16(cl, ba, gw1[to][ti]);
                if (ti >= 2) gw1[to][ti] = mfma16(ch, ld4(&T.m_lo[16 * (ti - 2) + c][4 * g]), gw1[to][ti]);
            }
        }
        __syncthreads();
    }
    // block sums: biases over the 16 cells of a lane group, then the waves in order
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            gb1[j] += __shfl_xor(gb1[j], o, 64);
            gb2[j] += __shfl_xor(gb2[j], o, 64);
            if (TOP) gwd[j] += __shfl_xor(gwd[j], o, 64);
        }
    if (TOP) {
        gbd += __shfl_xor(gbd, 1, 64);
        gbd += __shfl_xor(gbd, 2, 64);
        gbd += __shfl_xor(gbd, 4, 64);
        gbd += __shfl_xor(gbd, 8, 64);
    }
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
            auto put = [&](int idx, float val) {
                if (w == 0) red[idx] = val;
                else red[idx] += val;
            };
#pragma unroll
            for (int to = 0; to < 2; ++to)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int out = 16 * to + 4 * g + k;
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) put(kNnW2 + out * 32 + 16 * ti + c, gw2[to][ti][k]);
#pragma unroll
                    for (int ti = 0; ti < 4; ++ti) put(kNnW1 + out * 64 + 16 * ti + c, gw1[to][ti][k]);
                }
            if (c == 0) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int f = nn_pi(8 * g + j);
                    put(kNnB1 + f, gb1[j]);
                    put(kNnB2 + f, gb2[j]);
                    if (TOP) put(kNnLayerSize + f, gwd[j]);
                }
                if (TOP && g == 0) put(kNnLayerSize + 32, gbd);
            }
        }
        __syncthreads();
    }
    float* out = B.partial + int64_t(blockIdx.x) * kNnParams;
    const int base = kNnOffLayer + B.layer * kNnLayerSize;
    for (int k = threadIdx.x; k < kNnLayerSize; k += blockDim.x) out[base + k] = red[k];
    if (TOP)
        for (int k = threadIdx.x; k < 33; k += blockDim.x) out[kNnOffWd + k] = red[kNnLayerSize + k];
}

// Encoder: dh0 = base + 1/4 sum_j dam_j; dWe = dh0 x^T, dbe = dh0.
__global__ __launch_bounds__(256) void k_nn_enc_bwd(NnIn A, const float* base_in, const float* dam_in,
                                                     float* partial) {
    __shared__ float red[96];
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4, wv = threadIdx.x >> 6;
    const double isr = A.scal[SC_NN_INV_SR], isd = A.scal[SC_NN_INV_SD];
    float g0[8], g1[8], gb[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) g0[j] = g1[j] = gb[j] = 0.f;
    int64_t bg0, bg1;
    block_range((A.nc + 63) / 64, bg0, bg1);
    for (int64_t bg = bg0; bg < bg1; ++bg) {
        const int64_t i = bg * 64 + wv * 16 + c;
        if (i >= A.nc) continue;
        const int4 nb = A.nbr[i];
        const int nbs[4] = {nb.x, nb.y, nb.z, nb.w};
        float acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (nbs[k] < 0) continue;
            const float* q = dam_in + int64_t(nbs[k]) * 32 + 8 * g;
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += q[j];
        }
        const float* bq = base_in + i * 32 + 8 * g;
        const double r = double(A.r32[i]);
        const float x0 = float(r * isr), x1 = float(A.dinv[i] * r * isd);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float d = bq[j] + 0.25f * acc[j];
            g0[j] = fmaf(d, x0, g0[j]);
            g1[j] = fmaf(d, x1, g1[j]);
            gb[j] += d;
        }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            g0[j] += __shfl_xor(g0[j], o, 64);
            g1[j] += __shfl_xor(g1[j], o, 64);
            gb[j] += __shfl_xor(gb[j], o, 64);
        }
    for (int w = 0; w < 4; ++w) {
        if (wv == w && c == 0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int f = nn_pi(8 * g + j);
                if (w == 0) {
                    red[2 * f] = g0[j];
                    red[2 * f + 1] = g1[j];
                    red[64 + f] = gb[j];
                } else {
                    red[2 * f] += g0[j];
                    red[2 * f + 1] += g1[j];
                    red[64 + f] += gb[j];
                }
            }
        }
        __syncthreads();
    }
    float* out = partial + int64_t(blockIdx.x) * kNnParams;
    for (int k = threadIdx.x; k < 96; k += blockDim.x) out[kNnOffWe + k] = red[k];
}

// ---- losses ----------------------------------------------------------------------
// residual: res = r - K z, L = |res|^2 / |r|^2, w = K^T res, dy = -2 s_d / |r|^2 w
// energy:   a = K z, L = (z.a - 2 z.r) / r.D^-1 r, w = (a + K^T z) / 2 - r,
//           dy = 2 s_d / r.D^-1 r w
__device__ inline double row_dot(const Dev& d, const double* __restrict__ vals, const double* __restrict__ x,
                                 int64_t i) {
    const int64_t s = i >> 6;
    const int64_t base = d.k_off[s] + (i & 63);
    const int w = d.k_w[s];
    double y = d.k_diag[i] * x[i];
    for (int k = 0; k < w; ++k) {
        const int64_t at = base + int64_t(k) * 64;
        y += vals[at] * x[d.k_col[at]];
    }
    return y;
}

__global__ __launch_bounds__(256) void k_nn_resid(Dev d, const float* r32, const double* z, double* res) {
    __shared__ double lds[4];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double v = 0.0;
    if (i < d.nc) {
        const double e = double(r32[i]) - row_dot(d, d.k_val, z, i);
        res[i] = e;
        v = e * e;
    }
    const double s = block_sum256(v, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_nn_energy_a(Dev d, const float* r32, const double* z, double* a) {
    __shared__ double lds[4];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double v = 0.0;
    if (i < d.nc) {
        const double ai = row_dot(d, d.k_val, z, i);
        a[i] = ai;
        v = z[i] * ai - 2.0 * z[i] * double(r32[i]);
    }
    const double s = block_sum256(v, lds);
    if (threadIdx.x == 0) d.partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_nn_energy_w(Dev d, const double* kt, const float* r32, const double* z,
                                                     const double* a, double* w) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < d.nc) w[i] = 0.5 * (a[i] + row_dot(d, kt, z, i)) - double(r32[i]);
}

// loss of the step into *loss_slot and the factor of the top layer's dy
__global__ __launch_bounds__(1024) void k_nn_loss_fin(Dev d, int64_t nparts, int kind, double* loss_slot) {
    __shared__ double lds[16];
    const double s = reduce_partials_sum(d.partial, nparts, lds);
    if (threadIdx.x == 0) {
        double* sc = d.scal;
        const double sd = sc[SC_NN_SD];
        if (kind == 0) {
            const double rr = sc[SC_NN_RR];
            *loss_slot = rr > 0.0 ? s / rr : 0.0;
            sc[SC_NN_DSCALE] = rr > 0.0 ? -2.0 * sd / rr : 0.0;
        } else {
            const double rdr = sc[SC_NN_RDR];
            *loss_slot = rdr > 0.0 ? s / rdr : 0.0;
            sc[SC_NN_DSCALE] = rdr > 0.0 ? 2.0 * sd / rdr : 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void k_nn_spmv_t(Dev d, const double* kt, const double* x, double* y) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < d.nc) y[i] = row_dot(d, kt, x, i);
}

// ---- scales of the input ------------------------------------------------------
template <bool R32>
__global__ __launch_bounds__(256) void k_nn_scale(Dev d, const double* r64, const float* r32) {
    __shared__ double lds[4];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double a = 0.0, b = 0.0, e = 0.0;
    if (i < d.nc) {
        const double r = R32 ? double(r32[i]) : r64[i];
        const double q = d.k_dinv[i] * r;
        a = r * r;
        b = q * q;
        e = q * r;
    }
    const double s0 = block_sum256(a, lds);
    const double s1 = block_sum256(b, lds);
    const double s2 = block_sum256(e, lds);
    if (threadIdx.x == 0) {
        d.partial[blockIdx.x] = s0;
        d.partial[gridDim.x + blockIdx.x] = s1;
        d.partial[2 * gridDim.x + blockIdx.x] = s2;
    }
}

__device__ inline void set_scales(double* sc, double rr, double dd, int64_t n) {
    const double s_r = sqrt(rr / double(n)), s_d = sqrt(dd / double(n));
    sc[SC_NN_RR] = rr;
    sc[SC_NN_DD] = dd;
    sc[SC_NN_INV_SR] = s_r > 0.0 ? 1.0 / s_r : 0.0;
    sc[SC_NN_INV_SD] = s_d > 0.0 ? 1.0 / s_d : 0.0;
    sc[SC_NN_SD] = s_d;
}

__global__ __launch_bounds__(1024) void k_nn_scale_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    const double rr = reduce_partials_sum(d.partial, nparts, lds);
    const double dd = reduce_partials_sum(d.partial + nparts, nparts, lds);
    const double rdr = reduce_partials_sum(d.partial + 2 * nparts, nparts, lds);
    if (threadIdx.x == 0) {
        set_scales(d.scal, rr, dd, d.nc);
        d.scal[SC_NN_RDR] = rdr;
    }
}

// ---- gradient sum over blocks and Adam --------------------------------------------
// The gradient is the sum of the per-block sums, in two fixed-order stages:
// chunk c of kNnGradChunks adds blocks c, c + chunks, c + 2 chunks, ... (one
// thread per parameter and chunk, so many loads are in flight), then the
// Adam kernel adds the chunks in order.  Deterministic for a fixed grid.
__global__ __launch_bounds__(256) void k_nn_grad_chunks(NnDev n, int nblocks) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (p >= kNnParams) return;
    float g = 0.f;
    for (int b = c; b < nblocks; b += kNnGradChunks) g += n.partial[int64_t(b) * kNnParams + p];
    n.partial2[int64_t(c) * kNnParams + p] = g;
}

__global__ __launch_bounds__(256) void k_nn_adam(NnDev n, int apply, float lr, float c1, float c2,
                                                  float beta1, float beta2, float eps) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNnParams) return;
    float g = 0.f;
#pragma unroll
    for (int c = 0; c < kNnGradChunks; ++c) g += n.partial2[int64_t(c) * kNnParams + p];
    n.grad[p] = g;
    if (!apply) return;
    const float m = beta1 * n.adam_m[p] + (1.f - beta1) * g;
    const float v = beta2 * n.adam_v[p] + (1.f - beta2) * g * g;
    n.adam_m[p] = m;
    n.adam_v[p] = v;
    n.params[p] -= lr * (m * c1) / (sqrtf(v) * c2 + eps);
}

// ---- operand packing from the FP32 master copy ------------------------------------
__device__ inline __bf16 to_bf(float f) { return __builtin_bit_cast(__bf16, uint16_t(f2bf(f))); }

__global__ __launch_bounds__(256) void k_nn_pack(NnDev n) {
    const float* p = n.params;
    NnPack* P = n.pack;
    const int tid = threadIdx.x;
    for (int q = tid; q < 32; q += 256) {
        const int f = nn_pi(q);
        P->we0[q] = rbf(p[kNnOffWe + 2 * f]);
        P->we1[q] = rbf(p[kNnOffWe + 2 * f + 1]);
        P->be[q] = p[kNnOffBe + f];
        P->wd[q] = p[kNnOffWd + f];
    }
    if (tid == 0) P->bd = p[kNnOffBd];
    for (int l = 0; l < kNnLayers; ++l) {
        const float* W1 = p + kNnOffLayer + l * kNnLayerSize + kNnW1;   // [32][64]
        const float* W2 = p + kNnOffLayer + l * kNnLayerSize + kNnW2;   // [32][32]
        const float* b1 = p + kNnOffLayer + l * kNnLayerSize + kNnB1;
        const float* b2 = p + kNnOffLayer + l * kNnLayerSize + kNnB2;
        NnPackLayer& L = P->layer[l];
        for (int q = tid; q < 32; q += 256) {
            L.b1[q] = b1[nn_pi(q)];
            L.b2[q] = b2[nn_pi(q)];
        }
        // one thread per (fragment, lane): lane = e % 64, g = lane / 16, row = lane % 16
        for (int e = tid; e < 12 * 64; e += 256) {
            const int frag = e >> 6, lane = e & 63, g = lane >> 4, row = lane & 15;
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = nn_pi(8 * g + j);
                float w;
                if (frag < 4) {              // w1[t][s]; the m-half (s = 1) scaled by 1/4 (exact)
                    const int t = frag >> 1, s = frag & 1;
                    w = W1[(16 * t + row) * 64 + 32 * s + k];
                    if (s == 1) w = rbf(w) * 0.25f;
                } else if (frag < 6) {       // w2[t]
                    w = W2[(16 * (frag - 4) + row) * 32 + k];
                } else if (frag < 8) {       // w2t[t]
                    w = W2[k * 32 + 16 * (frag - 6) + row];
                } else {                     // w1t[t]
                    w = W1[k * 64 + 16 * (frag - 8) + row];
                }
                v[j] = to_bf(w);
            }
            if (frag < 4) L.w1[frag >> 1][frag & 1][lane] = v;
            else if (frag < 6) L.w2[frag - 4][lane] = v;
            else if (frag < 8) L.w2t[frag - 6][lane] = v;
            else L.w1t[frag - 8][lane] = v;
        }
    }
}

// ---- per-state set-up ---------------------------------------------------------------
// face neighbours from the cell->face table (-1 across a boundary face)
__global__ __launch_bounds__(256) void k_nn_neighbours(Dev d, int4* nbr) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= d.nc) return;
    int o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int code = d.c2f[k * d.nc + i];
        const int f = code >= 0 ? code : ~code;
        const int other = d.fL[f] == i ? d.fR[f] : d.fL[f];
        o[k] = other < d.nc ? other : -1;
    }
    nbr[i] = make_int4(o[0], o[1], o[2], o[3]);
}

// values of K^T in K's (symmetric) pattern: entry (i, j) takes K's (j, i);
// a missing mirror entry sets *flag
__global__ __launch_bounds__(256) void k_nn_transpose(Dev d, double* kt, int32_t* flag) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= d.nc) return;
    const int64_t s = i >> 6;
    const int64_t base = d.k_off[s] + (i & 63);
    const int w = d.k_w[s], len = d.k_len[i];
    for (int k = 0; k < w; ++k) {
        const int64_t at = base + int64_t(k) * 64;
        double v = 0.0;
        if (k < len) {
            const int64_t j = d.k_col[at];
            const int64_t sj = j >> 6;
            const int64_t bj = d.k_off[sj] + (j & 63);
            int lo = 0, hi = d.k_len[j] - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (d.k_col[bj + int64_t(mid) * 64] < i) lo = mid + 1;
                else hi = mid;
            }
            const int64_t atj = bj + int64_t(lo) * 64;
            if (hi >= 0 && d.k_col[atj] == i) v = d.k_val[atj];
            else *flag = 1;
        }
        kt[at] = v;
    }
}

// ---- flexible CG ------------------------------------------------------------------
// r = b - K x (kx: K x computed matrix-free, or null for the stored K);
// partial rr, bb, dd
__global__ __launch_bounds__(256) void k_fcg_setup(Dev d, const double* __restrict__ kx) {
    __shared__ double lds[4];
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (i < d.nc) {
        const double bi = d.b[i];
        const double ri = bi - (kx ? kx[i] : row_dot(d, d.k_val, d.x, i));
        d.r[i] = ri;
        const double q = d.k_dinv[i] * ri;
        a = ri * ri;
        b = bi * bi;
        c = q * q;
    }
    const double s0 = block_sum256(a, lds), s1 = block_sum256(b, lds), s2 = block_sum256(c, lds);
    if (threadIdx.x == 0) {
        d.partial[blockIdx.x] = s0;
        d.partial[gridDim.x + blockIdx.x] = s1;
        d.partial[2 * gridDim.x + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(1024) void k_fcg_setup_fin(Dev d, int64_t nparts, double tol, int maxit, int restart,
                                                        int fresh) {
    __shared__ double lds[16];
    const double rr = reduce_partials_sum(d.partial, nparts, lds);
    const double bb = reduce_partials_sum(d.partial + nparts, nparts, lds);
    const double dd = reduce_partials_sum(d.partial + 2 * nparts, nparts, lds);
    if (threadIdx.x == 0) {
        double* sc = d.scal;
        sc[SC_RR] = rr;
        sc[SC_TRUE_RR] = rr;
        sc[SC_BB] = bb;
        if (fresh) {
            sc[SC_TOL2BB] = tol * tol * bb;
            sc[SC_MAXIT] = double(maxit);
            sc[SC_RESTART] = double(restart);
            sc[SC_IT] = 0.0;
        }
        sc[SC_SINCE] = 0.0;
        sc[SC_DONE] = (rr <= sc[SC_TOL2BB] || bb == 0.0) ? 1.0 : (sc[SC_IT] >= sc[SC_MAXIT] ? 2.0 : 0.0);
        set_scales(sc, rr, dd, d.nc);
    }
}

// after the network: rz = z . r, p = z
__global__ __launch_bounds__(1024) void k_fcg_rz_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    if (d.scal[SC_DONE] != 0.0) return;
    const double zr = reduce_partials_sum(d.partial, nparts, lds);
    if (threadIdx.x == 0) d.scal[SC_RZ] = zr;
}

__global__ __launch_bounds__(256) void k_fcg_p0(Dev d) {
    if (d.scal[SC_DONE] != 0.0) return;
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < d.nc) d.p[i] = d.z[i];
}

// x += alpha p; r_old = r; r -= alpha q; partial rr, dd
__global__ __launch_bounds__(256) void k_fcg_axpy(Dev d, double* r_old) {
    __shared__ double lds[4];
    if (d.scal[SC_DONE] != 0.0) return;
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double a = 0.0, c = 0.0;
    if (i < d.nc) {
        const double alpha = d.scal[SC_ALPHA];
        d.x[i] = d.x[i] + alpha * d.p[i];
        const double ro = d.r[i];
        const double ri = ro - alpha * d.q[i];
        r_old[i] = ro;
        d.r[i] = ri;
        const double q = d.k_dinv[i] * ri;
        a = ri * ri;
        c = q * q;
    }
    const double s0 = block_sum256(a, lds), s1 = block_sum256(c, lds);
    if (threadIdx.x == 0) {
        d.partial[blockIdx.x] = s0;
        d.partial[gridDim.x + blockIdx.x] = s1;
    }
}

// count; convergence (1), limit (2) or a scheduled restart (3); input scales
__global__ __launch_bounds__(1024) void k_fcg_rr_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    double* sc = d.scal;
    if (sc[SC_DONE] != 0.0) return;
    const double rr = reduce_partials_sum(d.partial, nparts, lds);
    const double dd = reduce_partials_sum(d.partial + nparts, nparts, lds);
    if (threadIdx.x == 0) {
        sc[SC_RR] = rr;
        sc[SC_IT] = sc[SC_IT] + 1.0;
        sc[SC_SINCE] = sc[SC_SINCE] + 1.0;
        if (rr <= sc[SC_TOL2BB]) sc[SC_DONE] = 1.0;
        else if (sc[SC_IT] >= sc[SC_MAXIT]) sc[SC_DONE] = 2.0;
        else if (sc[SC_RESTART] > 0.0 && sc[SC_SINCE] >= sc[SC_RESTART]) sc[SC_DONE] = 3.0;
        set_scales(sc, rr, dd, d.nc);
    }
}

// flexible (Polak-Ribiere) beta = z_new . (r_new - r_old) / (z_old . r_old)
__global__ __launch_bounds__(1024) void k_fcg_beta_fin(Dev d, int64_t nparts) {
    __shared__ double lds[16];
    double* sc = d.scal;
    if (sc[SC_DONE] != 0.0) return;
    const double zr = reduce_partials_sum(d.partial, nparts, lds);
    const double zro = reduce_partials_sum(d.partial + nparts, nparts, lds);
    if (threadIdx.x == 0) {
        sc[SC_ZR] = zr;
        sc[SC_ZRO] = zro;
        sc[SC_BETA] = (zr - zro) / sc[SC_RZ];
        sc[SC_RZ] = zr;
    }
}

// training sample: out = r / s_r (FP32) after r = b - K x and its scales
__global__ __launch_bounds__(256) void k_nn_sample_out(Dev d, float* out) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < d.nc) out[i] = float(d.r[i] * d.scal[SC_NN_INV_SR]);
}

__global__ __launch_bounds__(256) void k_fcg_copy(int64_t n, const double* src, double* dst) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

inline unsigned rows256(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

// ---- launchers ------------------------------------------------------------------------
hipError_t launch_nn_pack(const NnDev& n, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_pack, dim3(1), dim3(256), 0, s, n);
    return hipGetLastError();
}

hipError_t launch_nn_neighbours(const Dev& d, const NnStateDev& a, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_neighbours, dim3(rows256(d.nc)), dim3(256), 0, s, d, a.nbr);
    return hipGetLastError();
}

hipError_t launch_nn_transpose(const Dev& d, const NnStateDev& a, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_transpose, dim3(rows256(d.nc)), dim3(256), 0, s, d, a.kt_val, a.flag);
    return hipGetLastError();
}

hipError_t launch_nn_scale(const Dev& d, const double* r64, const float* r32, hipStream_t s) {
    const unsigned nb = rows256(d.nc);
    if (r32) hipLaunchKernelGGL(k_nn_scale<true>, dim3(nb), dim3(256), 0, s, d, r64, r32);
    else hipLaunchKernelGGL(k_nn_scale<false>, dim3(nb), dim3(256), 0, s, d, r64, r32);
    hipLaunchKernelGGL(k_nn_scale_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb));
    return hipGetLastError();
}

static NnIn make_in(const Dev& d, const NnDev& n, const NnStateDev& a, const double* r64, const float* r32) {
    NnIn in;
    in.nc = d.nc;
    in.nbr = a.nbr;
    in.r64 = r64;
    in.r32 = r32;
    in.dinv = d.k_dinv;
    in.scal = d.scal;
    in.pack = n.pack;
    return in;
}

hipError_t launch_nn_layer(const Dev& d, const NnDev& n, const NnStateDev& a, int layer, const double* r64,
                           const float* r32, double* z, bool keep_h3, bool fcg, hipStream_t s) {
    NnFwd F;
    F.in = make_in(d, n, a, r64, r32);
    F.layer = layer;
    F.hin = layer == 0 ? nullptr : (layer == 1 ? a.h1 : a.h2);
    F.hout = layer == 0 ? a.h1 : (layer == 1 ? a.h2 : a.h3);
    F.z = z;
    F.r_old = a.r_old;
    F.partial = d.partial;
    const dim3 grid(nn_fwd_grid(d.nc)), block(256);
    const bool r32in = r32 != nullptr;
#define NN_L(K, R, C, KP) hipLaunchKernelGGL((k_nn_layer<K, R, C, KP>), grid, block, 0, s, F)
    if (layer == 0) {
        if (r32in) NN_L(0, true, false, false);
        else if (fcg) NN_L(0, false, true, false);
        else NN_L(0, false, false, false);
    } else if (layer == 1) {
        if (r32in) NN_L(1, true, false, false);
        else if (fcg) NN_L(1, false, true, false);
        else NN_L(1, false, false, false);
    } else {
        if (r32in) {
            if (keep_h3) NN_L(2, true, false, true);
            else NN_L(2, true, false, false);
        } else if (fcg) NN_L(2, false, true, false);
        else NN_L(2, false, false, false);
    }
#undef NN_L
    return hipGetLastError();
}

int nn_forward_grid(int64_t nc) { return nn_fwd_grid(nc); }

hipError_t launch_nn_backward(const Dev& d, const NnDev& n, const NnStateDev& a, const float* r32, int kind,
                              double* loss_slot, hipStream_t s) {
    // z in d.z; scratch in d.q; w in d.p
    const unsigned nb = rows256(d.nc);
    if (kind == 0) {
        hipLaunchKernelGGL(k_nn_resid, dim3(nb), dim3(256), 0, s, d, r32, d.z, d.q);
        hipLaunchKernelGGL(k_nn_loss_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb), 0, loss_slot);
        hipLaunchKernelGGL(k_nn_spmv_t, dim3(nb), dim3(256), 0, s, d, a.kt_val, d.q, d.p);
    } else {
        hipLaunchKernelGGL(k_nn_energy_a, dim3(nb), dim3(256), 0, s, d, r32, d.z, d.q);
        hipLaunchKernelGGL(k_nn_loss_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb), 1, loss_slot);
        hipLaunchKernelGGL(k_nn_energy_w, dim3(nb), dim3(256), 0, s, d, a.kt_val, r32, d.z, d.q, d.p);
    }
    NnBwd B;
    B.in = make_in(d, n, a, nullptr, r32);
    B.partial = n.partial;
    B.w = d.p;
    const dim3 grid(nn_bwd_grid(d.nc)), block(256);
    // last layer: input h2, output h3 -> base, dam0
    B.layer = 2; B.hin = a.h2; B.hout = a.h3; B.base_in = nullptr; B.dam_in = nullptr;
    B.base_out = a.base; B.dam_out = a.dam0;
    hipLaunchKernelGGL((k_nn_bwd<false, true>), grid, block, 0, s, B);
    // middle layer: input h1; base in place, dam0 -> dam1
    B.layer = 1; B.hin = a.h1; B.hout = nullptr; B.base_in = a.base; B.dam_in = a.dam0;
    B.base_out = a.base; B.dam_out = a.dam1;
    hipLaunchKernelGGL((k_nn_bwd<false, false>), grid, block, 0, s, B);
    // first layer: input re-encoded from r; dam1 -> dam0
    B.layer = 0; B.hin = nullptr; B.base_in = a.base; B.dam_in = a.dam1;
    B.base_out = a.base; B.dam_out = a.dam0;
    hipLaunchKernelGGL((k_nn_bwd<true, false>), grid, block, 0, s, B);
    hipLaunchKernelGGL(k_nn_enc_bwd, grid, block, 0, s, B.in, a.base, a.dam0, n.partial);
    return hipGetLastError();
}

int nn_backward_grid(int64_t nc) { return nn_bwd_grid(nc); }

hipError_t launch_nn_adam(const NnDev& n, int nblocks, int apply, float lr, float c1, float c2, float beta1,
                          float beta2, float eps, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_grad_chunks, dim3((kNnParams + 255) / 256, kNnGradChunks), dim3(256), 0, s, n, nblocks);
    hipLaunchKernelGGL(k_nn_adam, dim3((kNnParams + 255) / 256), dim3(256), 0, s, n, apply, lr, c1, c2,
                       beta1, beta2, eps);
    if (apply) hipLaunchKernelGGL(k_nn_pack, dim3(1), dim3(256), 0, s, n);
    return hipGetLastError();
}

hipError_t launch_nn_sample(const Dev& d, float* out, hipStream_t s) {
    const unsigned nb = rows256(d.nc);
    hipLaunchKernelGGL(k_fcg_setup, dim3(nb), dim3(256), 0, s, d, (const double*)nullptr);   // r = b - K x (partials unused)
    hipLaunchKernelGGL(k_nn_scale<false>, dim3(nb), dim3(256), 0, s, d, d.r, nullptr);
    hipLaunchKernelGGL(k_nn_scale_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb));
    hipLaunchKernelGGL(k_nn_sample_out, dim3(nb), dim3(256), 0, s, d, out);
    return hipGetLastError();
}

hipError_t launch_fcg_setup(const Dev& d, double tol, int maxit, int restart, bool fresh, hipStream_t s,
                            const double* kx) {
    const unsigned nb = rows256(d.nc);
    hipLaunchKernelGGL(k_fcg_setup, dim3(nb), dim3(256), 0, s, d, kx);
    hipLaunchKernelGGL(k_fcg_setup_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb), tol, maxit, restart,
                       fresh ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fcg_setup_tail(const Dev& d, const NnStateDev& a, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_rz_fin, dim3(1), dim3(1024), 0, s, d, nn_forward_parts(d, a));
    hipLaunchKernelGGL(k_fcg_p0, dim3(rows256(d.nc)), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_fcg_axpy(const Dev& d, const NnStateDev& a, hipStream_t s) {
    const unsigned nb = rows256(d.nc);
    hipLaunchKernelGGL(k_fcg_axpy, dim3(nb), dim3(256), 0, s, d, a.r_old);
    hipLaunchKernelGGL(k_fcg_rr_fin, dim3(1), dim3(1024), 0, s, d, int64_t(nb));
    return hipGetLastError();
}

hipError_t launch_fcg_beta(const Dev& d, const NnStateDev& a, hipStream_t s) {
    hipLaunchKernelGGL(k_fcg_beta_fin, dim3(1), dim3(1024), 0, s, d, nn_forward_parts(d, a));
    return hipGetLastError();
}

int64_t nn_forward_parts(const Dev& d, const NnStateDev& a) {
    return (a.tiles && a.fused) ? a.tiles->ntiles : int64_t(nn_fwd_grid(d.nc));
}

hipError_t launch_nn_fused(const Dev& d, const NnDev& n, const NnStateDev& a, const double* r64, double* z,
                           bool fcg, hipStream_t s) {
    const NnTiles& t = *a.tiles;
    NnFused F;
    F.in = make_in(d, n, a, r64, nullptr);
    F.ext_off = a.t_ext_off;
    F.ring = a.t_ring;
    F.cell = a.t_cell;
    F.nb_off = a.t_nb_off;
    F.nb = a.t_nb;
    F.ntiles = t.ntiles;
    F.ext_max = t.ext_max;
    F.z = z;
    F.r_old = a.r_old;
    F.partial = d.partial;
    const dim3 grid(unsigned((t.ntiles + 7) / 8 * 8)), block(256);
    const size_t lds = nn_fused_lds(t);
    if (fcg) hipLaunchKernelGGL(k_nn_fused<true>, grid, block, lds, s, F);
    else hipLaunchKernelGGL(k_nn_fused<false>, grid, block, lds, s, F);
    return hipGetLastError();
}

hipError_t setup_nn_fused(size_t lds) {
    if (lds <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nn_fused<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nn_fused<false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    return e;
}

hipError_t launch_fcg_backup(const Dev& d, const NnStateDev& a, bool restore, hipStream_t s) {
    if (restore) hipLaunchKernelGGL(k_fcg_copy, dim3(rows256(d.nc)), dim3(256), 0, s, d.nc, a.x_bak, d.x);
    else hipLaunchKernelGGL(k_fcg_copy, dim3(rows256(d.nc)), dim3(256), 0, s, d.nc, d.x, a.x_bak);
    return hipGetLastError();
}

}  // namespace mifvm
