// FP64 kernels of block GMRES (Sec. 2.4 names block variants of GMRES as a
// way to lower the iteration count): the products of a block Krylov basis
// with a block of at most 16 new vectors.
//
// Vectors are complex128 of length N, vector i of a basis at Q + i * qld.
//   k_bdots_partial / k_bdots_final:  C = Q^H W  (m x q, q <= 16), a GEMM with
//       the long dimension N as contraction, on the FP64 matrix cores;
//       two-stage with a fixed summation order, so bitwise reproducible.
//   k_bcombine:  X_c = beta X_c + alpha sum_i Q_i C(i, c)  (the Gram-Schmidt
//       update, the triangular change of basis and the solution update),
//       streaming over N with the block of X in registers.
#include "devtypes.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace hsw {

using C64 = Cx<double>;

// Each workgroup covers BD_CHUNK consecutive entries and 64 basis vectors
// (four 16-row tiles); its four waves take interleaved 16-entry blocks and
// their 16 x 16 tiles are summed through LDS.
constexpr int BD_CHUNK = 4096;

__global__ __launch_bounds__(256) void k_bdots_partial(const C64* __restrict__ Q, int64_t qld, int m,
                                                       const C64* __restrict__ W, int64_t wld, int q,
                                                       int64_t N, C64* __restrict__ partial) {
    __shared__ double red[3][4][2][4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int l16 = lane & 15, lk = lane >> 4;
    const int i0 = blockIdx.y * 64;
    const int64_t n0 = (int64_t)blockIdx.x * BD_CHUNK;
    md4 accR[4], accI[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        accR[t] = md4{0, 0, 0, 0};
        accI[t] = md4{0, 0, 0, 0};
    }
    const bool wcol = l16 < q;
    const C64* wp = W + (int64_t)l16 * wld;
    for (int blk = wave; blk < BD_CHUNK / 16; blk += 4) {
        const int64_t nb = n0 + (int64_t)blk * 16;
        if (nb >= N) break;
        // lane group lk supplies contraction index lk of each step s: entry nb + 4 lk + s
        const int64_t ne = nb + 4 * lk;
        C64 w[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            w[s] = (wcol && ne + s < N) ? wp[ne + s] : cx<double>(0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = i0 + 16 * t + l16;
            const bool qrow = i < m;
            const C64* qp = Q + (int64_t)i * qld;
            C64 a[4];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                a[s] = (qrow && ne + s < N) ? qp[ne + s] : cx<double>(0, 0);
            // (ar - i ai)(wr + i wi) = (ar wr + ai wi) + i (ar wi - ai wr)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                accR[t] = mfma4(a[s].re, w[s].re, accR[t]);
                accR[t] = mfma4(a[s].im, w[s].im, accR[t]);
                accI[t] = mfma4(a[s].re, w[s].im, accI[t]);
                accI[t] = mfma4(-a[s].im, w[s].re, accI[t]);
            }
        }
    }
    if (wave > 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                red[wave - 1][t][0][r][lane] = accR[t][r];
                red[wave - 1][t][1][r][lane] = accI[t][r];
            }
    }
    __syncthreads();
    if (wave != 0) return;
    const int nchunk_stride = m * q;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double re = accR[t][r], im = accI[t][r];
            for (int w = 0; w < 3; ++w) {
                re += red[w][t][0][r][lane];
                im += red[w][t][1][r][lane];
            }
            const int i = i0 + 16 * t + mfma_out_row<double>(lk, r);
            if (i < m && l16 < q)
                partial[(int64_t)blockIdx.x * nchunk_stride + (int64_t)i * q + l16] = cx<double>(re, im);
        }
}

// out[i * q + c] = sum over chunks of partial, in chunk order.
__global__ __launch_bounds__(256) void k_bdots_final(const C64* __restrict__ partial, int nchunk,
                                                     int mq, C64* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= mq) return;
    C64 t = cx<double>(0, 0);
    for (int c = 0; c < nchunk; ++c) t = t + partial[(int64_t)c * mq + e];
    out[e] = t;
}

// X_c = beta X_c + alpha sum_{i < m} Q_i C(i, c) for c < q (X_c at X + col[c] * ld,
// or c * ld without col).  Each thread owns one entry n of every column and
// reads all of its inputs before it writes, so X may be part of Q.
__global__ __launch_bounds__(256) void k_bcombine(const C64* Q, int64_t qld, int m,
                                                  const C64* __restrict__ C, int q, C64* X, int64_t ld,
                                                  const int* __restrict__ col, int64_t N, double alpha,
                                                  double beta) {
    __shared__ C64 sc[64 * 16];
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    C64 acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = cx<double>(0, 0);
    for (int i0 = 0; i0 < m; i0 += 64) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < 64 * 16; idx += 256) {
            const int r = idx >> 4, c = idx & 15;
            sc[idx] = (i0 + r < m && c < q) ? C[(int64_t)(i0 + r) * q + c] : cx<double>(0, 0);
        }
        __syncthreads();
        if (n < N) {
            const int iend = m - i0 < 64 ? m - i0 : 64;
            for (int r = 0; r < iend; ++r) {
                const C64 v = Q[(int64_t)(i0 + r) * qld + n];
#pragma unroll
                for (int c = 0; c < 16; ++c) cfma(acc[c], v, sc[r * 16 + c]);
            }
        }
    }
    if (n >= N) return;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        if (c < q) {
            C64* xp = X + (int64_t)(col ? col[c] : c) * ld + n;
            const C64 add = scale(acc[c], alpha);
            *xp = beta == 0.0 ? add : scale(*xp, beta) + add;
        }
    }
}

// ---------------------------------------------------------------------------
int bdots_chunks(int64_t N) { return (int)((N + BD_CHUNK - 1) / BD_CHUNK); }

void launch_bdots(const C64* Q, int64_t qld, int m, const C64* W, int64_t wld, int q, int64_t N,
                  C64* partial, C64* out, hipStream_t st) {
    const int nch = bdots_chunks(N);
    HSW_LAUNCH(k_bdots_partial, dim3(nch, (m + 63) / 64), dim3(256), 0, st, Q, qld, m, W, wld, q, N,
               partial);
    HSW_LAUNCH(k_bdots_final, dim3((m * q + 255) / 256), dim3(256), 0, st, (const C64*)partial, nch,
               m * q, out);
}

void launch_bcombine(const C64* Q, int64_t qld, int m, const C64* C, int q, C64* X, int64_t ld,
                     const int* col, int64_t N, double alpha, double beta, hipStream_t st) {
    HSW_LAUNCH(k_bcombine, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, Q, qld, m, C, q, X, ld,
               col, N, alpha, beta);
}

}  // namespace hsw
