// Batched multifrontal partial LDL^T of the panels' auxiliary problems
// (Sec. 2.2) and the selectively inverted fronts used by the solves.
//
// Every launch covers all fronts of one elimination-tree depth over all
// panels and problems; a flat work list of (front instance, tile or block)
// pairs maps workgroups to work, so fronts of uneven size share a launch.
//
// Front storage.  A front with s pivots and u update rows is the
// (s+u) x (s+u) lower triangle F = [F_TL *; F_BL F_BR].  Its first s columns
// [F_TL; F_BL] live in the persistent factor buffer as an (s+u) x s
// column-major block (leading dimension s+u); F_BR (u x u, column-major)
// lives in a workspace indexed by the parity of the depth, kept until the
// parent has pulled it (extend-add) one level up.
#include <utility>

#include "devtypes.hpp"
#include "kernels.hpp"
#include "mfma.hpp"
#include "stencil.hpp"

namespace hsw {

__device__ inline void tri_decode_dev(int t, int& ti, int& tj) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
}

template <typename T>
__device__ inline Cx<T>* front_at(Cx<T>* L, Cx<T>* W, int n, int s, int u, int i, int j) {
    return j < s ? L + (int64_t)j * n + i : W + (int64_t)(j - s) * u + (i - s);
}

// A box node's coordinates (a1, a2, q) of box index a1 + a2 Nx + q Nx Ny,
// packed 16 bits each (panel boxes are far below 65536 nodes per axis).
__device__ inline uint64_t box_coords(const PanelDev& P, int b) {
    const int NxNy = P.Nx * P.Ny;
    const int q = b / NxNy, r = b - q * NxNy, a2 = r / P.Nx, a1 = r - a2 * P.Nx;
    return (uint64_t)(uint32_t)a1 | ((uint64_t)(uint32_t)a2 << 16) | ((uint64_t)(uint32_t)q << 32);
}

// Entry H(bi, bj) of a panel's auxiliary operator between box nodes with
// packed coordinates ci, cj (box_coords); zero when they are not stencil
// neighbours.
__device__ inline Cx<double> aux_entry(const ProbDev& Q, const PanelDev& P, const Cx<double>* et,
                                       uint64_t ci, uint64_t cj, Cx<double> kappa2, double inv_h2) {
    const int a1i = (int)(ci & 0xffff), a2i = (int)((ci >> 16) & 0xffff), qi = (int)(ci >> 32);
    const int a1j = (int)(cj & 0xffff), a2j = (int)((cj >> 16) & 0xffff), qj = (int)(cj >> 32);
    const Cx<double>* e3n = et + P.e3_off;
    const Cx<double>* ie3 = et + P.e3_off + P.nz;
    if (ci == cj) {
        NodeStretch st = node_stretch(Q, et, a1i, a2i, e3n, ie3, qi);
        double c = velocity_at(Q, a1i, a2i, P.lo - P.ga + qi);
        return diag_entry(st, c, kappa2, inv_h2);
    }
    int d1 = a1i - a1j, d2 = a2i - a2j, d3 = qi - qj;
    int ad = abs(d1) + abs(d2) + abs(d3);
    if (ad != 1) return cx<double>(0.0, 0.0);
    int ax = d1 != 0 ? 0 : (d2 != 0 ? 1 : 2);
    int sgn = d1 + d2 + d3;  // +1: i is the upper node
    int la1 = sgn > 0 ? a1j : a1i, la2 = sgn > 0 ? a2j : a2i, lq = sgn > 0 ? qj : qi;
    return coupling_entry(Q, et, e3n, ie3, la1, la2, lq, ax, inv_h2);
}

// ---------------------------------------------------------------------------
// Front assembly: original entries of H_i in the pivot columns plus the
// extend-add of the children's update matrices (pulled, fixed order: no
// atomics, bitwise deterministic).  One workgroup per 64 x 64 lower tile.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const int2* __restrict__ work,
                                                  const FrontInst* __restrict__ inst,
                                                  const PanelDev* __restrict__ pan,
                                                  const ProbDev* __restrict__ prob,
                                                  const int* __restrict__ perm,
                                                  const int* __restrict__ ulist,
                                                  const int* __restrict__ cmap,
                                                  const Cx<double>* __restrict__ et,
                                                  Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ Wcur,
                                                  const Cx<T>* __restrict__ Wchild) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    int ti, tj;
    tri_decode_dev(w.y, ti, tj);
    const int r0 = ti * TILE, c0 = tj * TILE;
    __shared__ int rpos[2][TILE], cpos[2][TILE];
    __shared__ uint64_t rbox[TILE], cbox[TILE];  // box coordinates (box_coords) of the rows and columns
    const int tid = threadIdx.x;
    const PanelDev P = pan[f.panel];
    if (tid < 2 * TILE) {
        const bool isrow = tid < TILE;
        const int l = isrow ? tid : tid - TILE;
        const int i = (isrow ? r0 : c0) + l;
        uint64_t bx = 0;
        int p0 = -1, p1 = -1;
        if (i < n) {
            int e = i < f.s ? f.start + i : ulist[f.uoff + i - f.s];
            bx = box_coords(P, perm[P.perm_off + e]);
            if (f.child0 >= 0) p0 = cmap[f.moff + i];
            if (f.child1 >= 0) p1 = cmap[f.moff + n + i];
        }
        if (isrow) { rbox[l] = bx; rpos[0][l] = p0; rpos[1][l] = p1; }
        else { cbox[l] = bx; cpos[0][l] = p0; cpos[1][l] = p1; }
    }
    __syncthreads();
    const ProbDev Q = prob[P.prob];
    const Cx<double> kappa2 = kappa_sq(Q, Q.alpha);
    const double inv_h2 = 1.0 / (Q.h * Q.h);
    int64_t cw[2] = {0, 0};
    int cu[2] = {0, 0};
    if (f.child0 >= 0) { cw[0] = inst[f.child0].woff; cu[0] = inst[f.child0].u; }
    if (f.child1 >= 0) { cw[1] = inst[f.child1].woff; cu[1] = inst[f.child1].u; }
    Cx<T>* L = Lb + f.loff;
    Cx<T>* W = Wcur + f.woff;
    for (int idx = tid; idx < TILE * TILE; idx += 256) {
        const int li = idx & (TILE - 1), lj = idx / TILE;
        const int i = r0 + li, j = c0 + lj;
        if (i >= n || j >= n || i < j) continue;
        Cx<T> acc = cx<T>(0, 0);
        if (j < f.s) acc = ccast<T>(aux_entry(Q, P, et, rbox[li], cbox[lj], kappa2, inv_h2));
        for (int ch = 0; ch < 2; ++ch) {
            int pi = rpos[ch][li], pj = cpos[ch][lj];
            if (pi >= 0 && pj >= 0) acc = acc + Wchild[cw[ch] + (int64_t)pj * cu[ch] + pi];
        }
        *front_at(L, W, n, f.s, f.u, i, j) = acc;
    }
}

constexpr int LDP = 64 + 4;  // padded row length of the planar LDS tiles

// acc += R C^T over KC columns for the 64 x 64 tile rows x cols: R (rows) and
// C (cols) are planar LDS tiles [k][row]; wave w owns the 32 x 32 quadrant
// (rows (w&1)*32, cols (w>>1)*32) as 2 x 2 blocks of 16 x 16.  In block
// (bi, bj), lane l and register r hold tile row (w&1)*32 + 16 bi + (l&15)
// and tile column (w>>1)*32 + 16 bj + mfma_out_row<T>(l>>4, r).
template <typename T, int KC>
__device__ inline void tile_cgemm(typename MfmaAcc<T>::type (&are)[2][2],
                                  typename MfmaAcc<T>::type (&aim)[2][2], const T (*Rre)[LDP],
                                  const T (*Rim)[LDP], const T (*Cre)[LDP], const T (*Cim)[LDP],
                                  int kmax) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int li = l & 15, lk = l >> 4;
#pragma unroll 2
    for (int kk = 0; kk < KC; kk += 4) {
        if (kk >= kmax) break;
        T cr[2], ci[2], rr[2], ri[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            cr[q] = Cre[kk + lk][wc + 16 * q + li];
            ci[q] = Cim[kk + lk][wc + 16 * q + li];
            rr[q] = Rre[kk + lk][wr + 16 * q + li];
            ri[q] = Rim[kk + lk][wr + 16 * q + li];
        }
        // four rounds of eight independent products, so that no product
        // waits for the previous one on the same accumulator
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                are[bi][bj] = mfma4(cr[bj], rr[bi], are[bi][bj]);
                aim[bi][bj] = mfma4(cr[bj], ri[bi], aim[bi][bj]);
            }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                are[bi][bj] = mfma4(-ci[bj], ri[bi], are[bi][bj]);
                aim[bi][bj] = mfma4(ci[bj], rr[bi], aim[bi][bj]);
            }
    }
}

// The same tile product with each complex product as three real ones (the
// three-multiplication form): with C = a + ib and R = c + id, k1 += (a + b) c,
// k2 += a (d - c) and k3 += b (c + d); the product's real part is k1 - k3, its
// imaginary part k1 + k2 (cgemm64_pipe folds them in).  A quarter fewer
// matrix-core products for one more accumulator block per 16 x 16 block.
template <typename T, int KC>
__device__ inline void tile_cgemm3(typename MfmaAcc<T>::type (&k1)[2][2],
                                   typename MfmaAcc<T>::type (&k2)[2][2],
                                   typename MfmaAcc<T>::type (&k3)[2][2], const T (*Rre)[LDP],
                                   const T (*Rim)[LDP], const T (*Cre)[LDP], const T (*Cim)[LDP],
                                   int kmax) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int li = l & 15, lk = l >> 4;
#pragma unroll 2
    for (int kk = 0; kk < KC; kk += 4) {
        if (kk >= kmax) break;
        T cr[2], ci[2], rr[2], ri[2], cs[2], rd[2], rs[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            cr[q] = Cre[kk + lk][wc + 16 * q + li];
            ci[q] = Cim[kk + lk][wc + 16 * q + li];
            rr[q] = Rre[kk + lk][wr + 16 * q + li];
            ri[q] = Rim[kk + lk][wr + 16 * q + li];
            cs[q] = cr[q] + ci[q];
            rd[q] = ri[q] - rr[q];
            rs[q] = rr[q] + ri[q];
        }
        // three rounds of four independent products
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) k1[bi][bj] = mfma4(cs[bj], rr[bi], k1[bi][bj]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) k2[bi][bj] = mfma4(cr[bj], rd[bi], k2[bi][bj]);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) k3[bi][bj] = mfma4(ci[bj], rs[bi], k3[bi][bj]);
    }
}

// acc += R C^T over k < K for a 64 x 64 tile, R and C read from memory by
// ldR(k, row) and ldC(k, col) in chunks of KC columns.  Software pipelined:
// the loads of chunk c + 1 are in flight while chunk c runs on the matrix
// cores from one of two LDS buffers, so one barrier per chunk suffices.
// CT picks the thread mapping of the C loads: false, consecutive threads read
// consecutive cols (contiguous when C is stored [k][col]); true, consecutive
// k (contiguous when C is stored [col][k]).  M3 takes the three-product tile
// (tile_cgemm3), for the callers whose occupancy its extra accumulators do
// not lower.  Ends with a barrier (except for K <= 0, which returns at once);
// the caller's LDS buffers are free afterwards.
template <typename T, int KC, bool CT = false, bool M3 = false, typename LR, typename LC>
__device__ inline void cgemm64_pipe(typename MfmaAcc<T>::type (&are)[2][2],
                                    typename MfmaAcc<T>::type (&aim)[2][2], int K, LR ldR, LC ldC,
                                    T (*Rre)[KC][LDP], T (*Rim)[KC][LDP], T (*Cre)[KC][LDP],
                                    T (*Cim)[KC][LDP]) {
    constexpr int PER = KC * 64 / 256;
    const int tid = threadIdx.x;
    const int nch = (K + KC - 1) / KC;
    if (nch <= 0) return;
    Cx<T> r[PER], c[PER];
    auto cmap_ = [](int idx, int& a, int& m) {
        if (CT) {
            m = idx % KC;
            a = idx / KC;
        } else {
            a = idx & 63;
            m = idx >> 6;
        }
    };
    // k of a thread's R entries: (tid >> 6) + 4 q, the same across a wave
    // (so the bounds tests are uniform branches and a loader's per-k values,
    // such as the pivot d_k of the update's C operand, are scalar loads)
    const int wq = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q, a = tid & 63, kk = k0 + wq + 4 * q;
            r[q] = kk < K ? ldR(kk, a) : cx<T>(0, 0);
            int ca, cm;
            if (CT) {
                cmap_(idx, ca, cm);
            } else {
                ca = a;
                cm = wq + 4 * q;
            }
            c[q] = k0 + cm < K ? ldC(k0 + cm, ca) : cx<T>(0, 0);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q, a = idx & 63, m = idx >> 6;
            Rre[buf][m][a] = r[q].re;
            Rim[buf][m][a] = r[q].im;
            int ca, cm;
            cmap_(idx, ca, cm);
            Cre[buf][cm][ca] = c[q].re;
            Cim[buf][cm][ca] = c[q].im;
        }
    };
    fetch(0);
    put(0);
    __syncthreads();
    if constexpr (M3) {
        // the three-product accumulators start from the incoming sums:
        // re = k1 - k3 and im = k1 + k2 with k1 = 0, k2 = im, k3 = -re
        typename MfmaAcc<T>::type k1[2][2], k2[2][2], k3[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                k1[bi][bj] = typename MfmaAcc<T>::type{0, 0, 0, 0};
                k2[bi][bj] = aim[bi][bj];
                k3[bi][bj] = -are[bi][bj];
            }
        for (int ch = 0; ch < nch; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nch) fetch((ch + 1) * KC);
            tile_cgemm3<T, KC>(k1, k2, k3, Rre[buf], Rim[buf], Cre[buf], Cim[buf], K - ch * KC);
            if (ch + 1 < nch) put(buf ^ 1);
            __syncthreads();
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                are[bi][bj] = k1[bi][bj] - k3[bi][bj];
                aim[bi][bj] = k1[bi][bj] + k2[bi][bj];
            }
    } else {
        for (int ch = 0; ch < nch; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nch) fetch((ch + 1) * KC);
            tile_cgemm<T, KC>(are, aim, Rre[buf], Rim[buf], Cre[buf], Cim[buf], K - ch * KC);
            if (ch + 1 < nch) put(buf ^ 1);
            __syncthreads();
        }
    }
}

// acc += R C^T over k < K for a 64 x 64 tile whose R operand is already in
// LDS as planar [k][row] tiles (Rre, Rim, at least K rows); only C, read by
// ldC(k, col) with consecutive threads on consecutive cols, is staged (as in
// cgemm64_pipe: chunks of KC, the next chunk's loads in flight during this
// one's products), and each complex product is three real ones
// (tile_cgemm3).  Ends with a barrier (except for K <= 0).
template <typename T, int KC, typename LC>
__device__ inline void cgemm64_rlds(typename MfmaAcc<T>::type (&are)[2][2],
                                    typename MfmaAcc<T>::type (&aim)[2][2], int K, const T (*Rre)[LDP],
                                    const T (*Rim)[LDP], LC ldC, T (*Cre)[KC][LDP], T (*Cim)[KC][LDP]) {
    constexpr int PER = KC * 64 / 256;
    const int tid = threadIdx.x;
    const int nch = (K + KC - 1) / KC;
    if (nch <= 0) return;
    const int wq = __builtin_amdgcn_readfirstlane(tid >> 6);
    Cx<T> c[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int m = wq + 4 * q;
            c[q] = k0 + m < K ? ldC(k0 + m, tid & 63) : cx<T>(0, 0);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            Cre[buf][wq + 4 * q][tid & 63] = c[q].re;
            Cim[buf][wq + 4 * q][tid & 63] = c[q].im;
        }
    };
    typename MfmaAcc<T>::type k1[2][2], k2[2][2], k3[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            k1[bi][bj] = typename MfmaAcc<T>::type{0, 0, 0, 0};
            k2[bi][bj] = aim[bi][bj];
            k3[bi][bj] = -are[bi][bj];
        }
    fetch(0);
    put(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) fetch((ch + 1) * KC);
        tile_cgemm3<T, KC>(k1, k2, k3, Rre + ch * KC, Rim + ch * KC, Cre[buf], Cim[buf], K - ch * KC);
        if (ch + 1 < nch) put(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            are[bi][bj] = k1[bi][bj] - k3[bi][bj];
            aim[bi][bj] = k1[bi][bj] + k2[bi][bj];
        }
}

// ---------------------------------------------------------------------------
// The same 64 x 64 tile product with complex BF16 inputs on the BF16 matrix
// cores (16 x 16 x 16 products, FP32 accumulation): the operands are rounded
// to bf16 (nearest even) as they are staged, chunk by chunk of 16 k, in LDS
// tiles [row][k] (k contiguous: lane l reads the four k = 4 (l/16) + 0..3 of
// row l % 16 in one access, the bf16 instruction's operand layout).  The
// output layout of the 16 x 16 blocks is that of the FP32 product, so
// tile_cgemm's accumulators and the callers' epilogues serve both.
typedef short bf4 __attribute__((ext_vector_type(4)));
constexpr int BK = 16, BKP = BK + 4;  // chunk of k, padded row length of the bf16 tiles

__device__ inline unsigned short bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);  // inf / nan kept
    return (unsigned short)(u >> 16);
}

__device__ inline mf4 mfma_bf16(bf4 a, bf4 b, mf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ inline void tile_cgemm_bf16(mf4 (&are)[2][2], mf4 (&aim)[2][2],
                                       const unsigned short (*R)[64][BKP], const unsigned short (*C)[64][BKP]) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int li = l & 15, lk = l >> 4;
    bf4 cr[2], ci[2], cn[2], rr[2], ri[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        cr[q] = *reinterpret_cast<const bf4*>(&C[0][wc + 16 * q + li][4 * lk]);
        ci[q] = *reinterpret_cast<const bf4*>(&C[1][wc + 16 * q + li][4 * lk]);
        rr[q] = *reinterpret_cast<const bf4*>(&R[0][wr + 16 * q + li][4 * lk]);
        ri[q] = *reinterpret_cast<const bf4*>(&R[1][wr + 16 * q + li][4 * lk]);
        cn[q] = ci[q] ^ (bf4)(short)0x8000;  // -C_im: the sign bits flipped
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            are[bi][bj] = mfma_bf16(cr[bj], rr[bi], are[bi][bj]);
            aim[bi][bj] = mfma_bf16(cr[bj], ri[bi], aim[bi][bj]);
        }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            are[bi][bj] = mfma_bf16(cn[bj], ri[bi], are[bi][bj]);
            aim[bi][bj] = mfma_bf16(ci[bj], rr[bi], aim[bi][bj]);
        }
}

// acc += R C^T over k < K, as cgemm64_pipe (same loaders, same pipelining:
// chunk c + 1 in flight while chunk c runs from the other LDS buffer), with
// the operands rounded to bf16 and multiplied on the BF16 matrix cores.
template <typename LR, typename LC>
__device__ inline void cgemm64_pipe_bf16(mf4 (&are)[2][2], mf4 (&aim)[2][2], int K, LR ldR, LC ldC,
                                         unsigned short (*R)[2][64][BKP], unsigned short (*C)[2][64][BKP]) {
    constexpr int PER = BK * 64 / 256;
    const int tid = threadIdx.x;
    const int nch = (K + BK - 1) / BK;
    if (nch <= 0) return;
    Cx<float> r[PER], c[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q, a = idx & 63, kk = k0 + (idx >> 6);
            r[q] = kk < K ? ldR(kk, a) : cx<float>(0, 0);
            c[q] = kk < K ? ldC(kk, a) : cx<float>(0, 0);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + 256 * q, a = idx & 63, m = idx >> 6;
            R[buf][0][a][m] = bf16_bits(r[q].re);
            R[buf][1][a][m] = bf16_bits(r[q].im);
            C[buf][0][a][m] = bf16_bits(c[q].re);
            C[buf][1][a][m] = bf16_bits(c[q].im);
        }
    };
    fetch(0);
    put(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) fetch((ch + 1) * BK);
        tile_cgemm_bf16(are, aim, R[buf], C[buf]);
        if (ch + 1 < nch) put(buf ^ 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 16 x 16 complex tile product on the matrix cores, acc += A B over k < K
// (K <= 16): lane l supplies A(l % 16, k) and B(k, l % 16) for k = kk + l / 16;
// register r of lane l then holds row mfma_out_row<T>(l / 16, r), column l % 16.
template <typename T, typename GA, typename GB>
__device__ inline void cmma16(typename MfmaAcc<T>::type& are, typename MfmaAcc<T>::type& aim, int K,
                              GA getA, GB getB) {
    const int l = threadIdx.x & 63;
    const int i = l & 15, kq = l >> 4;
    for (int kk = 0; kk < K; kk += 4) {
        const int kx = kk + kq;
        const Cx<T> a = kx < K ? getA(i, kx) : cx<T>(0, 0);
        const Cx<T> b = kx < K ? getB(kx, i) : cx<T>(0, 0);
        are = mfma4(a.re, b.re, are);
        aim = mfma4(a.re, b.im, aim);
        are = mfma4(-a.im, b.im, are);
        aim = mfma4(a.im, b.re, aim);
    }
}

template <typename T>
__device__ inline Cx<T> shfl_cx(Cx<T> v, int src) {
    return cx<T>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

// The value of lane L (a compile-time constant) in every lane, read through a
// scalar register (no LDS round trip, unlike a shuffle).
__device__ inline float lane_bcast(float v, int L) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}
__device__ inline double lane_bcast(double v, int L) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), L);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), L);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ inline Cx<T> lane_bcast_cx(Cx<T> v, int L) {
    return cx<T>(lane_bcast(v.re, L), lane_bcast(v.im, L));
}

// Reciprocal of a pivot: a power-of-two prescale keeps |b|^2 in range; in
// FP32 the hardware reciprocal (about one ulp) replaces the division.
__device__ inline Cx<float> pivot_recip(Cx<float> b) {
    const int e = __builtin_amdgcn_frexp_expf(fmaxf(fabsf(b.re), fabsf(b.im)));
    const float br = ldexpf(b.re, -e), bi = ldexpf(b.im, -e);
    const float r = __builtin_amdgcn_rcpf(br * br + bi * bi);
    return cx<float>(ldexpf(br * r, -e), ldexpf(-bi * r, -e));
}
__device__ inline Cx<double> pivot_recip(Cx<double> b) { return crecip(b); }

// Lane m of each 16-lane row, in every lane of that row (DPP row broadcast:
// a register move, no LDS round trip).
template <int m>
__device__ inline float row_bcast(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x150 + m, 0xf, 0xf, false));
}
template <int m, typename T>
__device__ inline Cx<T> row_bcast_cx(Cx<T> v) {
    return cx<T>(row_bcast<m>(v.re), row_bcast<m>(v.im));
}

// Step m of the complex64 16 x 16 sub-block factorisation (see diag16); m is
// a template parameter so that every register index is static.  The whole
// trailing square is updated, so it stays symmetric: the operands A(j, m)
// and X(m, j) of lane (i, j) are then both held by lane (m, j) of its own row
// of 16 lanes, and reach it by a row broadcast.
template <int m, typename T>
__device__ inline void diag16_step(Cx<T> (&a)[4], Cx<T> (&x)[4], int i, int jg, int l, Cx<T>& dl,
                                   Cx<T>& idl) {
    constexpr int src = 16 * (m & 3);  // lanes holding column m: l / 16 == m % 4, register m / 4
    const Cx<T> d = lane_bcast_cx(a[m >> 2], m + src);  // the pivot, from one fixed lane
    const Cx<T> idm = pivot_recip(d);
    const Cx<T> aim = shfl_cx(a[m >> 2], i + src);
    const Cx<T> li = aim * idm;
    const bool below = i > m;
    // every operand is read before any register of this step changes: the
    // lanes holding column m overwrite it with l_im below
    Cx<T> amj[4], xm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        amj[q] = row_bcast_cx<m>(a[q]);  // A(m, j) = A(j, m)
        xm[q] = row_bcast_cx<m>(x[q]);   // X(m, j), final at step m
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        Cx<T> na = a[q], nx = x[q];
        cfms(na, li, amj[q]);
        cfms(nx, li, xm[q]);
        a[q] = (below && j > m) ? na : a[q];
        x[q] = (below && j <= m) ? nx : x[q];
        a[q] = (below && j == m) ? li : a[q];
    }
    // lane m keeps the pivot and its reciprocal
    dl = l == m ? d : dl;
    idl = l == m ? idm : idl;
}

template <typename T, int... M>
__device__ inline void diag16_steps(std::integer_sequence<int, M...>, Cx<T> (&a)[4], Cx<T> (&x)[4], int i,
                                    int jg, int l, Cx<T>& dl, Cx<T>& idl) {
    (diag16_step<M, T>(a, x, i, jg, l, dl, idl), ...);
}

// One wave factors the 16 x 16 diagonal sub-block at c0 (w <= 16 valid
// columns; the rest is padded with the identity) and inverts its unit lower
// factor.  Lane l holds rows i = l % 16 at columns j = l / 16 + 4q of the
// block and of X; the 16 steps are unrolled and free of branches.  The block
// is read whole (the upper part from its symmetric lower entries).
template <typename T>
__device__ inline void diag16(T (*Mre)[LDP], T (*Mim)[LDP], Cx<T>* dv, Cx<T>* __restrict__ dinv,
                              int c0, int w, int* bad) {
    const int l = threadIdx.x & 63;
    const int i = l & 15, jg = l >> 4;
    Cx<T> a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        const T one = i == j ? (T)1 : (T)0;
        const int r = i >= j ? i : j, c = i >= j ? j : i;
        a[q] = (i < w && j < w) ? cx<T>(Mre[c0 + c][c0 + r], Mim[c0 + c][c0 + r]) : cx<T>(one, 0);
        x[q] = cx<T>(one, 0);
    }
    Cx<T> dl = cx<T>(1, 0), idl = cx<T>(1, 0);
    diag16_steps<T>(std::make_integer_sequence<int, 16>{}, a, x, i, jg, l, dl, idl);
    // pivots and reciprocals of the block's columns; the first bad one is reported
    const bool mine = l < w;
    if (mine) {
        dv[c0 + l] = dl;
        dinv[c0 + l] = idl;
    }
    const bool finite = isfinite(dl.re) && isfinite(dl.im) && isfinite(idl.re) && isfinite(idl.im);
    const unsigned long long bm = __ballot(mine && (!finite || (dl.re == 0 && dl.im == 0)));
    if (l == 0 && bm != 0 && *bad < 0) *bad = c0 + __ffsll((long long)bm) - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        if (i < w && j < w && i >= j) {
            Mre[c0 + j][c0 + i] = a[q].re;
            Mim[c0 + j][c0 + i] = a[q].im;
        }
        if (i < w && j < w && i > j) {  // X(i, j) in the upper triangle: row j, column i
            Mre[c0 + i][c0 + j] = x[q].re;
            Mim[c0 + i][c0 + j] = x[q].im;
        }
    }
}

// The complex128 form of the sub-block factorisation: the operands of a step
// arrive by cross-lane shuffles.  (With row broadcasts its register pressure
// spills inside the pivot loop: 8.4 against 17.4 ms at 50^3.)  Step m:
template <int m, typename T>
__device__ inline void diag16s_step(Cx<T> (&a)[4], Cx<T> (&x)[4], int i, int jg, int l, int c0, int w,
                                   Cx<T>* dv, Cx<T>* __restrict__ dinv, int& first_bad) {
    constexpr int src = 16 * (m & 3);  // lanes holding column m: l / 16 == m % 4, register m / 4
    const Cx<T> d = lane_bcast_cx(a[m >> 2], m + src);  // the pivot, from one fixed lane
    const Cx<T> idm = pivot_recip(d);
    const Cx<T> aim = shfl_cx(a[m >> 2], i + src);
    const Cx<T> li = aim * idm;
    const bool below = i > m;
    // every operand is read before any register of this step changes: the
    // lanes holding column m overwrite it with l_im below
    Cx<T> ajm[4], xm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ajm[q] = shfl_cx(a[m >> 2], jg + 4 * q + src);  // A(j, m)
        xm[q] = shfl_cx(x[q], m + 16 * jg);             // X(m, j), final at step m
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        Cx<T> na = a[q], nx = x[q];
        cfms(na, li, ajm[q]);
        cfms(nx, li, xm[q]);
        const bool ua = below && j > m && j <= i, ux = below && j <= m;
        a[q] = ua ? na : a[q];
        x[q] = ux ? nx : x[q];
        a[q] = (below && j == m) ? li : a[q];
    }
    if (l == 0 && m < w) {
        dv[c0 + m] = d;
        dinv[c0 + m] = idm;
        const bool finite = isfinite(d.re) && isfinite(d.im) && isfinite(idm.re) && isfinite(idm.im);
        if ((!finite || (d.re == 0 && d.im == 0)) && first_bad < 0) first_bad = c0 + m;
    }
}

template <typename T, int... M>
__device__ inline void diag16s_steps(std::integer_sequence<int, M...>, Cx<T> (&a)[4], Cx<T> (&x)[4], int i,
                                    int jg, int l, int c0, int w, Cx<T>* dv, Cx<T>* __restrict__ dinv,
                                    int& first_bad) {
    (diag16s_step<M, T>(a, x, i, jg, l, c0, w, dv, dinv, first_bad), ...);
}

// One wave factors the 16 x 16 diagonal sub-block at c0 (w <= 16 valid
// columns; the rest is padded with the identity) and inverts its unit lower
// factor.  Lane l holds rows i = l % 16 at columns j = l / 16 + 4q of the
// block and of X; the 16 steps are unrolled and free of branches.
template <typename T>
__device__ inline void diag16s(T (*Mre)[LDP], T (*Mim)[LDP], Cx<T>* dv, Cx<T>* __restrict__ dinv,
                              int c0, int w, int* bad) {
    const int l = threadIdx.x & 63;
    const int i = l & 15, jg = l >> 4;
    Cx<T> a[4], x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        const T one = i == j ? (T)1 : (T)0;
        a[q] = (i >= j && i < w) ? cx<T>(Mre[c0 + j][c0 + i], Mim[c0 + j][c0 + i]) : cx<T>(one, 0);
        x[q] = cx<T>(one, 0);
    }
    int first_bad = -1;
    diag16s_steps<T>(std::make_integer_sequence<int, 16>{}, a, x, i, jg, l, c0, w, dv, dinv, first_bad);
    if (l == 0 && first_bad >= 0 && *bad < 0) *bad = first_bad;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = jg + 4 * q;
        if (i < w && j < w && i >= j) {
            Mre[c0 + j][c0 + i] = a[q].re;
            Mim[c0 + j][c0 + i] = a[q].im;
        }
        if (i < w && j < w && i > j) {  // X(i, j) in the upper triangle: row j, column i
            Mre[c0 + i][c0 + j] = x[q].re;
            Mim[c0 + i][c0 + j] = x[q].im;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ldlt_diag(const int2* __restrict__ work,
                                                   const FrontInst* __restrict__ inst,
                                                   Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ dinv,
                                                   int k, int* __restrict__ err) {
    typedef typename MfmaAcc<T>::type V4;
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    const int b = min(NB, f.s - k);
    Cx<T>* L = Lb + f.loff + (int64_t)k * n + k;  // block origin, leading dimension n
    __shared__ T Mre[NB][LDP], Mim[NB][LDP];      // M[col][row]
    __shared__ T Tre[4][16][17], Tim[4][16][17];  // per-wave 16 x 16 scratch
    __shared__ Cx<T> dv[NB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    if (tid == 0) bad = -1;
    constexpr int LB = sizeof(T) == 4 ? 16 : 8;  // loads in flight per thread
#pragma unroll
    for (int q0 = 0; q0 < NB * NB / 256; q0 += LB) {
        Cx<T> v[LB];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int idx = tid + 256 * (q0 + q), row = idx & (NB - 1), col = idx / NB;
            const bool in = row < b && col < b && row >= col;
            v[q] = L[in ? (int64_t)col * n + row : 0];
            if (!in) v[q] = cx<T>(0, 0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int idx = tid + 256 * (q0 + q), row = idx & (NB - 1), col = idx / NB;
            Mre[col][row] = v[q].re;
            Mim[col][row] = v[q].im;
        }
    }
    __syncthreads();
    const int nJ = (b + 15) / 16;
    for (int J = 0; J < nJ; ++J) {
        const int c0 = 16 * J, wj = min(16, b - c0);
        if (wave == 0) {
            if constexpr (sizeof(T) == 4) diag16<T>(Mre, Mim, dv, dinv + f.doff + k, c0, wj, &bad);
            else diag16s<T>(Mre, Mim, dv, dinv + f.doff + k, c0, wj, &bad);
        }
        __syncthreads();
        const int r0 = c0 + wj, nr = b - r0;
        if (nr <= 0) continue;
        const int nt = (nr + 15) / 16;
        // rows below: L(r, c0+j) = dinv_j sum_m A(r, c0+m) X_JJ(j, m)
        for (int t = wave; t < nt; t += 4) {
            const int rt = r0 + 16 * t;
            V4 are = V4{0, 0, 0, 0}, aim = V4{0, 0, 0, 0};
            cmma16<T>(are, aim, wj,
                      [&](int ii, int m) { return rt + ii < b ? cx<T>(Mre[c0 + m][rt + ii], Mim[c0 + m][rt + ii]) : cx<T>(0, 0); },
                      [&](int m, int j) {
                          if (j >= wj || m > j) return cx<T>(0, 0);
                          if (m == j) return cx<T>(1, 0);
                          return cx<T>(Mre[c0 + j][c0 + m], Mim[c0 + j][c0 + m]);
                      });
            // all lanes have read their operands before any lane of the wave writes
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ii = mfma_out_row<T>(lk, r), j = li;
                if (rt + ii < b && j < wj) {
                    const Cx<T> v = cx<T>(are[r], aim[r]) * pivot_recip(dv[c0 + j]);
                    Mre[c0 + j][rt + ii] = v.re;
                    Mim[c0 + j][rt + ii] = v.im;
                }
            }
        }
        __syncthreads();
        // trailing lower tiles: A(i, j) -= sum_m L(i, c0+m) d_m L(j, c0+m)
        for (int t = wave; t < nt * (nt + 1) / 2; t += 4) {
            int ti, tj;
            tri_decode_dev(t, ti, tj);
            const int ri = r0 + 16 * ti, cj = r0 + 16 * tj;
            V4 are = V4{0, 0, 0, 0}, aim = V4{0, 0, 0, 0};
            cmma16<T>(are, aim, wj,
                      [&](int ii, int m) { return ri + ii < b ? cx<T>(Mre[c0 + m][ri + ii], Mim[c0 + m][ri + ii]) : cx<T>(0, 0); },
                      [&](int m, int j) {
                          return cj + j < b ? cx<T>(Mre[c0 + m][cj + j], Mim[c0 + m][cj + j]) * dv[c0 + m] : cx<T>(0, 0);
                      });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = ri + mfma_out_row<T>(lk, r), gj = cj + li;
                if (gi < b && gj < b && gi >= gj) {
                    Mre[gj][gi] -= are[r];
                    Mim[gj][gi] -= aim[r];
                }
            }
        }
        __syncthreads();
    }
    // off-diagonal blocks of X = L^{-1}; X(r, c) with r > c lives at M[r][c]
    for (int I = 1; I < nJ; ++I) {
        const int i0 = 16 * I;
        for (int J = wave; J < I; J += 4) {
            const int j0 = 16 * J;
            V4 tre = V4{0, 0, 0, 0}, tim = V4{0, 0, 0, 0};
            for (int K = J; K < I; ++K) {
                const int k0 = 16 * K;
                cmma16<T>(tre, tim, 16,
                          [&](int ii, int kk) {  // L(i0+ii, k0+kk)
                              return i0 + ii < b && k0 + kk < b ? cx<T>(Mre[k0 + kk][i0 + ii], Mim[k0 + kk][i0 + ii]) : cx<T>(0, 0);
                          },
                          [&](int kk, int j) {  // X(k0+kk, j0+j)
                              const int r = k0 + kk, c = j0 + j;
                              if (r >= b || c >= b || r < c) return cx<T>(0, 0);
                              if (r == c) return cx<T>(1, 0);
                              return cx<T>(Mre[r][c], Mim[r][c]);
                          });
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Tre[wave][mfma_out_row<T>(lk, r)][li] = tre[r];
                Tim[wave][mfma_out_row<T>(lk, r)][li] = tim[r];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            V4 xre = V4{0, 0, 0, 0}, xim = V4{0, 0, 0, 0};
            cmma16<T>(xre, xim, 16,
                      [&](int ii, int kk) {  // X(i0+ii, i0+kk)
                          const int r = i0 + ii, c = i0 + kk;
                          if (r >= b || c >= b || r < c) return cx<T>(0, 0);
                          if (r == c) return cx<T>(1, 0);
                          return cx<T>(Mre[r][c], Mim[r][c]);
                      },
                      [&](int kk, int j) { return cx<T>(Tre[wave][kk][j], Tim[wave][kk][j]); });
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gr = i0 + mfma_out_row<T>(lk, r), gc = j0 + li;
                if (gr < b && gc < b) {
                    Mre[gr][gc] = -xre[r];
                    Mim[gr][gc] = -xim[r];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int row = idx & (NB - 1), col = idx / NB;
        if (row < b && col < b) L[(int64_t)col * n + row] = cx<T>(Mre[col][row], Mim[col][row]);
    }
    if (tid == 0 && bad >= 0) {
        if (atomicCAS(&err[0], -1, w.x) == -1) err[1] = k + bad;
    }
}

// Panel rows below the diagonal block: F_BL := F_BL L_kk^{-T} D_kk^{-1} for 64
// rows per workgroup, as a product with the stored L_kk^{-1} on the matrix
// cores: X(r, j) = dinv_j sum_{m <= j} P(r, m) L_kk^{-1}(j, m).
template <typename T>
__global__ __launch_bounds__(256) void k_panel_trsm(const int2* __restrict__ work,
                                                    const FrontInst* __restrict__ inst,
                                                    Cx<T>* __restrict__ Lb,
                                                    const Cx<T>* __restrict__ dinv, int k) {
    constexpr int KC = 16;
    typedef typename MfmaAcc<T>::type V4;
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    const int b = min(NB, f.s - k);
    Cx<T>* L = Lb + f.loff;
    __shared__ T Rre[2][KC][LDP], Rim[2][KC][LDP], Cre[2][KC][LDP], Cim[2][KC][LDP];
    const int tid = threadIdx.x;
    const int rbeg = k + b + w.y * 64, rend = min(rbeg + 64, n);
    V4 are[2][2], aim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            are[bi][bj] = V4{0, 0, 0, 0};
            aim[bi][bj] = V4{0, 0, 0, 0};
        }
    // P(r, m) through a descriptor cut at the front's n x s block: rows past
    // rend read finite values that reach only rows never stored
    const BufRsrc rl = buf_rsrc(L, (uint32_t)n * f.s * (uint32_t)sizeof(Cx<T>));
    cgemm64_pipe<T, KC, true, true>(  // L_kk^{-1}(a, m) is contiguous in m: transposed C loads
        are, aim, b,
        [&](int m, int a) {
            Cx<T> v;
            BufCx<T>::load(rl, ((uint32_t)(k + m) * n + rbeg + a) * (uint32_t)sizeof(Cx<T>), v.re, v.im);
            return v;
        },
        [&](int m, int a) {
            // L_kk^{-1}(a, m): 1 on the diagonal, stored at L(k + m, k + a) when m < a
            if (a >= b || m > a) return cx<T>(0, 0);
            if (m == a) return cx<T>(1, 0);
            return L[(int64_t)(k + a) * n + k + m];
        },
        Rre, Rim, Cre, Cim);
    const int l = tid & 63, wv = tid >> 6;
    const int li = l & 15, lk = l >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rbeg + (wv & 1) * 32 + 16 * bi + li;
                const int j = (wv >> 1) * 32 + 16 * bj + mfma_out_row<T>(lk, r);
                if (row < rend && j < b)
                    L[(int64_t)(k + j) * n + row] = cx<T>(are[bi][bj][r], aim[bi][bj][r]) * dinv[f.doff + k + j];
            }
}

// ---------------------------------------------------------------------------
// Schur-complement updates of the fronts on the matrix cores (Sec. 2.2:
// F_BR := F_BR - Z F_BL^T, applied blockwise), F[i,j] -= sum_m L[i,m] d_m L[j,m]
// over the lower triangle, m in [kbeg, kbeg + K).  One workgroup per 64 x 64
// output tile; the modes differ in which tiles and which pivots:
//   UPD_TRAIL  right-looking: pivot block [k, k+b) into every later row and
//              column (tiles of the triangle from t0 = k + b), K = b;
//   UPD_LEFT   left-looking: every earlier pivot into block column [k, k+b)
//              (row tiles from k), K = k;
//   UPD_SCHUR  every pivot into F_BR (tiles of the triangle from s), K = s;
//   UPD_PIVOTS as UPD_TRAIL but only into the pivot columns (< s): F_BR is
//              left to one UPD_SCHUR at the end (the hybrid order).
// With bf16 != 0 the inputs are rounded to bfloat16 (a bf16-input,
// FP32-accumulate product).
enum { UPD_TRAIL = 0, UPD_LEFT = 1, UPD_SCHUR = 2, UPD_PIVOTS = 3 };

// Round to the nearest bfloat16 (ties to even), kept in an FP32 register:
// products of two such values are exact in FP32, so the matrix cores then
// compute a bf16-input, FP32-accumulate product.
__device__ inline float round_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}
__device__ inline double round_bf16(double x) { return x; }

// bf16: 0 complex products in the working precision; 1 complex BF16 inputs
// on the BF16 matrix cores (BF, complex64 only); 2 the same bf16-rounded
// inputs on the FP32 matrix cores.
// Complex64 without BF16 inputs takes the three-product tile and is held to
// 128 registers (4 waves per SIMD, which its LDS allows); complex128 keeps
// four products (its extra accumulator blocks would cost occupancy).
template <typename T, bool BF>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && !BF) ? 4 : 1) void k_update(const int2* __restrict__ work,
                                                const FrontInst* __restrict__ inst,
                                                Cx<T>* __restrict__ Lb, Cx<T>* __restrict__ Wcur,
                                                int k, int mode, int bf16) {
    constexpr int KC = 16;
    typedef typename MfmaAcc<T>::type V4;
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u;
    int kbeg, K, r0, c0, cend;
    if (mode == UPD_LEFT) {
        const int b = min(NB, f.s - k);
        kbeg = 0;
        K = k;
        r0 = k + 64 * w.y;
        c0 = k;
        cend = k + b;
    } else {
        const bool blockwise = mode != UPD_SCHUR;
        const int b = blockwise ? min(NB, f.s - k) : f.s;
        const int t0 = blockwise ? k + b : f.s;
        kbeg = blockwise ? k : 0;
        K = b;
        int ti, tj;
        tri_decode_dev(w.y, ti, tj);
        r0 = t0 + ti * TILE;
        c0 = t0 + tj * TILE;
        cend = mode == UPD_PIVOTS ? f.s : n;
    }
    Cx<T>* L = Lb + f.loff;
    Cx<T>* W = Wcur + f.woff;
    const int tid = threadIdx.x;
    const int l = tid & 63, wv = tid >> 6;
    const int li = l & 15, lk = l >> 4;
    // the output tile's current values, fetched while the product runs
    Cx<T> old[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = r0 + (wv & 1) * 32 + 16 * bi + li;
                const int j = c0 + (wv >> 1) * 32 + 16 * bj + mfma_out_row<T>(lk, r);
                old[bi][bj][r] = (i < n && j < cend && i >= j) ? *front_at(L, W, n, f.s, f.u, i, j)
                                                               : cx<T>(0, 0);
            }
    V4 are[2][2], aim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            are[bi][bj] = V4{0, 0, 0, 0};
            aim[bi][bj] = V4{0, 0, 0, 0};
        }
    // Operand loads through a descriptor cut at the end of the front's n x s
    // block: a row past n (or a column past cend) reads a finite value of the
    // block (or zero past its end) that only reaches output entries never
    // stored, so the loads need no per-lane test.
    const BufRsrc rl = buf_rsrc(L, (uint32_t)n * f.s * (uint32_t)sizeof(Cx<T>));
    auto ldR = [&](int m, int a) {
        Cx<T> v;
        BufCx<T>::load(rl, ((uint32_t)(kbeg + m) * n + r0 + a) * (uint32_t)sizeof(Cx<T>), v.re, v.im);
        return v;
    };
    auto ldC = [&](int m, int a) {  // L[j,m] d_m (the pivot is the same across a wave)
        const Cx<T>* col = L + (int64_t)(kbeg + m) * n;
        Cx<T> v;
        BufCx<T>::load(rl, ((uint32_t)(kbeg + m) * n + c0 + a) * (uint32_t)sizeof(Cx<T>), v.re, v.im);
        return v * col[kbeg + m];
    };
    if constexpr (BF) {
        // complex BF16 inputs on the BF16 matrix cores
        __shared__ unsigned short Rb[2][2][64][BKP], Cb[2][2][64][BKP];
        cgemm64_pipe_bf16(are, aim, K, ldR, ldC, Rb, Cb);
    } else {
        __shared__ T Rre[2][KC][LDP], Rim[2][KC][LDP], Cre[2][KC][LDP], Cim[2][KC][LDP];
        if (bf16) {
            // the same inputs rounded to bf16, multiplied on the FP32 matrix cores
            // (products of bf16 values are exact in FP32: the reference of the path above)
            auto rnd = [](Cx<T> v) { return cx<T>(round_bf16(v.re), round_bf16(v.im)); };
            cgemm64_pipe<T, KC>(
                are, aim, K, [&](int m, int a) { return rnd(ldR(m, a)); },
                [&](int m, int a) { return rnd(ldC(m, a)); }, Rre, Rim, Cre, Cim);
        } else {
            cgemm64_pipe<T, KC, false, sizeof(T) == 4>(are, aim, K, ldR, ldC, Rre, Rim, Cre, Cim);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = r0 + (wv & 1) * 32 + 16 * bi + li;
                const int j = c0 + (wv >> 1) * 32 + 16 * bj + mfma_out_row<T>(lk, r);
                if (i < n && j < cend && i >= j)
                    *front_at(L, W, n, f.s, f.u, i, j) = old[bi][bj][r] - cx<T>(are[bi][bj][r], aim[bi][bj][r]);
            }
}

// ---------------------------------------------------------------------------
// Selective inversion (Sec. 2.2): G = X with X L_F = [I; F_BL], i.e.
// G = [L_F^{-1}; F_BL L_F^{-1}], so that both multifrontal triangular solves
// of a front become one product with G.  Rows are independent: one
// workgroup per 64 rows, sweeping the 64-column pivot blocks from last to
// first:  acc = B_blk - X(:, later columns) L(later, blk)  and then
// X_blk = acc L_blk^{-1}, both on the matrix cores; L_blk^{-1} is the
// diagonal-block inverse the factorisation stored above the diagonal.  A
// block's columns depend only on later columns, so stopping the sweep at
// the front's first formed column g0 leaves the formed columns unchanged.
// Complex64 is held to 168 registers: with its 51 KB of LDS, three
// workgroups share a compute unit.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 3 : 1) void k_inverse(const int2* __restrict__ work,
                                                 const FrontInst* __restrict__ inst, const Cx<T>* Lb,
                                                 Cx<T>* Gb, Cx<T>* Tb) {
    constexpr int KC = 16;
    typedef typename MfmaAcc<T>::type V4;
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u, s = f.s;
    const Cx<T>* L = Lb + f.loff;
    Cx<T>* G = Gb + f.loff;
    // X(row, col): rows of L_F^{-1} in the depth's scratch (s x s, column-major)
    // when Tb is given, every other row (and all rows without Tb) in G.  With
    // Tb, G may be L itself: this workgroup's rows of F_BL are only read by
    // it, before they are overwritten, and the rows of L_F that every row
    // block reads are left in place.
    Cx<T>* TF = Tb ? Tb + f.toff : nullptr;
    auto xat = [&](int row, int col) -> Cx<T>* {
        return (TF && row < s) ? TF + (int64_t)col * s + row : G + (int64_t)col * n + row;
    };
    const int r0 = w.y * 64;
    const int tid = threadIdx.x;
    const int l = tid & 63, wv = tid >> 6;
    const int li = l & 15, lk = l >> 4;
    __shared__ T Cre[2][KC][LDP], Cim[2][KC][LDP];
    // the block accumulator [col][row] (Are, Aim), which the second product
    // takes as its R operand in place; the first product stages its R chunks
    // in the same memory (it ends before the accumulator is written)
    __shared__ T ubuf[2 * 64 * LDP];
    T(*Are)[LDP] = reinterpret_cast<T(*)[LDP]>(ubuf);
    T(*Aim)[LDP] = reinterpret_cast<T(*)[LDP]>(ubuf + 64 * LDP);
    T(*Rre)[KC][LDP] = reinterpret_cast<T(*)[KC][LDP]>(ubuf);
    T(*Rim)[KC][LDP] = reinterpret_cast<T(*)[KC][LDP]>(ubuf + 2 * KC * LDP);
    static_assert(4 * KC <= 2 * 64, "the first product's R buffers fit in the accumulator's memory");
    const int ncb = (s + 63) / 64;
    for (int cbk = ncb - 1; cbk >= f.g0 / 64; --cbk) {
        const int c0 = cbk * 64, c1 = min(c0 + 64, s), bw = c1 - c0;
        __syncthreads();  // the previous block's columns of G, stored by every thread, are read below
        if (r0 + 63 < c0) {  // rows of the identity above the block: zero in L_F^{-1}
            for (int idx = tid; idx < 64 * 64; idx += 256) {
                const int rr = idx & 63, cc = idx / 64;
                if (cc < bw && r0 + rr < n) *xat(r0 + rr, c0 + cc) = cx<T>(0, 0);
            }
            continue;
        }
        V4 are[2][2], aim[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                are[bi][bj] = V4{0, 0, 0, 0};
                aim[bi][bj] = V4{0, 0, 0, 0};
            }
        // sum over the later pivot columns m >= c1: X(rows, m) L(m, blk); L(m, c0 + a)
        // is contiguous in m, so its loads use the transposed mapping.  Rows of
        // L_F^{-1} are zero right of the diagonal, so a block of such rows stops
        // at its own last row.
        const int kend = r0 + 64 <= s ? r0 + 64 : s;
        cgemm64_pipe<T, KC, true, true>(
            are, aim, kend - c1,
            [&](int m, int a) { return r0 + a < n ? *xat(r0 + a, c1 + m) : cx<T>(0, 0); },
            [&](int m, int a) { return a < bw ? L[(int64_t)(c0 + a) * n + c1 + m] : cx<T>(0, 0); },
            Rre, Rim, Cre, Cim);
        // acc = B_blk - sum, into LDS as [col][row]
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = (wv & 1) * 32 + 16 * bi + li;
                    const int cc = (wv >> 1) * 32 + 16 * bj + mfma_out_row<T>(lk, r);
                    const int row = r0 + rr;
                    Cx<T> bv = cx<T>(0, 0);
                    if (cc < bw && row < n) {
                        if (row < s) bv = cx<T>(row == c0 + cc ? (T)1 : (T)0, 0);
                        else bv = L[(int64_t)(c0 + cc) * n + row];
                    }
                    Are[cc][rr] = bv.re - are[bi][bj][r];
                    Aim[cc][rr] = bv.im - aim[bi][bj][r];
                    are[bi][bj][r] = 0;
                    aim[bi][bj][r] = 0;
                }
        __syncthreads();
        // X_blk = acc L_blk^{-1}: X(r, j) = sum_{m >= j} acc(r, m) Linv(m, j)
        cgemm64_rlds<T, KC>(
            are, aim, bw, Are, Aim,
            [&](int m, int a) {
                // Linv(m, a) for m > a is stored at L(c0 + a, c0 + m) (upper triangle)
                if (a >= bw || m < a) return cx<T>(0, 0);
                if (m == a) return cx<T>(1, 0);
                return L[(int64_t)(c0 + m) * n + c0 + a];
            },
            Cre, Cim);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + (wv & 1) * 32 + 16 * bi + li;
                    const int cc = (wv >> 1) * 32 + 16 * bj + mfma_out_row<T>(lk, r);
                    if (cc < bw && row < n) *xat(row, c0 + cc) = cx<T>(are[bi][bj][r], aim[bi][bj][r]);
                }
    }
}

// L_F^{-1} from the depth's scratch over the L_F rows of the factor block
// (rows 64 w.y .. of every formed pivot column), after the depth's inversion.
template <typename T>
__global__ __launch_bounds__(256) void k_lf_copy(const int2* __restrict__ work,
                                                 const FrontInst* __restrict__ inst, Cx<T>* __restrict__ Lb,
                                                 const Cx<T>* __restrict__ Tb) {
    const int2 w = work[blockIdx.x];
    const FrontInst f = inst[w.x];
    const int n = f.s + f.u, s = f.s;
    const int r0 = w.y * 64;
    Cx<T>* L = Lb + f.loff;
    const Cx<T>* TF = Tb + f.toff;
    for (int idx = threadIdx.x; idx < 64 * (s - f.g0); idx += 256) {
        const int col = f.g0 + (idx >> 6), row = r0 + (idx & 63);
        if (row < s) L[(int64_t)col * n + row] = TF[(int64_t)col * s + row];
    }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_assemble(const int2* work, int nwork, const FrontInst* inst, const PanelDev* pan,
                     const ProbDev* prob, const int* perm, const int* ulist, const int* cmap,
                     const Cx<double>* et, Cx<T>* Lb, Cx<T>* Wcur, const Cx<T>* Wchild,
                     hipStream_t st) {
    if (nwork <= 0) return;
    HSW_LAUNCH(k_assemble<T>, dim3(nwork), dim3(256), 0, st, work, inst, pan, prob, perm,
                       ulist, cmap, et, Lb, Wcur, Wchild);
}
template <typename T>
void launch_ldlt_diag(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* dinv,
                      int k, int* err, hipStream_t st) {
    if (nwork <= 0) return;
    HSW_LAUNCH(k_ldlt_diag<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, dinv, k, err);
}
template <typename T>
void launch_panel_trsm(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb,
                       const Cx<T>* dinv, int k, hipStream_t st) {
    if (nwork <= 0) return;
    HSW_LAUNCH(k_panel_trsm<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, dinv, k);
}
template <typename T>
void launch_update(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, Cx<T>* Wcur, int k,
                   int mode, int bf16, hipStream_t st) {
    if (nwork <= 0) return;
    if constexpr (sizeof(T) == 4) {
        if (bf16 == 1) {
            HSW_LAUNCH((k_update<T, true>), dim3(nwork), dim3(256), 0, st, work, inst, Lb, Wcur, k, mode, bf16);
            return;
        }
    }
    HSW_LAUNCH((k_update<T, false>), dim3(nwork), dim3(256), 0, st, work, inst, Lb, Wcur, k, mode, bf16);
}
template <typename T>
void launch_inverse(const int2* work, int nwork, const FrontInst* inst, const Cx<T>* Lb, Cx<T>* Gb,
                    Cx<T>* Tb, hipStream_t st) {
    if (nwork <= 0) return;
    HSW_LAUNCH(k_inverse<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, Gb, Tb);
}
template <typename T>
void launch_lf_copy(const int2* work, int nwork, const FrontInst* inst, Cx<T>* Lb, const Cx<T>* Tb,
                    hipStream_t st) {
    if (nwork <= 0) return;
    HSW_LAUNCH(k_lf_copy<T>, dim3(nwork), dim3(256), 0, st, work, inst, Lb, Tb);
}

#define HSW_INST(T)                                                                              \
    template void launch_assemble<T>(const int2*, int, const FrontInst*, const PanelDev*,       \
                                     const ProbDev*, const int*, const int*, const int*,        \
                                     const Cx<double>*, Cx<T>*, Cx<T>*, const Cx<T>*,           \
                                     hipStream_t);                                              \
    template void launch_ldlt_diag<T>(const int2*, int, const FrontInst*, Cx<T>*, Cx<T>*, int,   \
                                      int*, hipStream_t);                                       \
    template void launch_panel_trsm<T>(const int2*, int, const FrontInst*, Cx<T>*, const Cx<T>*, \
                                       int, hipStream_t);                                       \
    template void launch_update<T>(const int2*, int, const FrontInst*, Cx<T>*, Cx<T>*, int, int,  \
                                   int, hipStream_t);                                           \
    template void launch_inverse<T>(const int2*, int, const FrontInst*, const Cx<T>*, Cx<T>*,    \
                                    Cx<T>*, hipStream_t);                                       \
    template void launch_lf_copy<T>(const int2*, int, const FrontInst*, Cx<T>*, const Cx<T>*,    \
                                    hipStream_t);
HSW_INST(float)
HSW_INST(double)
#undef HSW_INST

}  // namespace hsw
