// Types shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hsw {

// Interleaved complex number (re, im) in FP32 or FP64.
template <typename R>
struct __align__(2 * sizeof(R)) Cx {
    R re, im;
};

template <typename R>
__host__ __device__ inline Cx<R> cx(R re, R im) {
    Cx<R> z;
    z.re = re;
    z.im = im;
    return z;
}
template <typename R>
__host__ __device__ inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return cx<R>(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return cx<R>(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ inline Cx<R> operator-(Cx<R> a) { return cx<R>(-a.re, -a.im); }
template <typename R>
__host__ __device__ inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
    return cx<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ inline Cx<R> scale(Cx<R> a, R s) { return cx<R>(a.re * s, a.im * s); }
// acc += a * b
template <typename R>
__host__ __device__ inline void cfma(Cx<R>& acc, Cx<R> a, Cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc -= a * b
template <typename R>
__host__ __device__ inline void cfms(Cx<R>& acc, Cx<R> a, Cx<R> b) {
    acc.re = fma(-a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(-a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}
// conj(a) * b
template <typename R>
__host__ __device__ inline Cx<R> cjmul(Cx<R> a, Cx<R> b) {
    return cx<R>(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// 1 / b by the plain formula conj(b) / |b|^2, with a power-of-two prescale so
// that |b|^2 neither overflows nor underflows in the working precision.
template <typename R>
__host__ __device__ inline Cx<R> crecip(Cx<R> b) {
    R m = fmax(fabs(b.re), fabs(b.im));
    int e = 0;
    frexp(m, &e);
    R br = ldexp(b.re, -e), bi = ldexp(b.im, -e);
    R den = br * br + bi * bi;
    return cx<R>(ldexp(br / den, -e), ldexp(-bi / den, -e));
}
template <typename R>
__host__ __device__ inline Cx<R> cdiv(Cx<R> a, Cx<R> b) { return a * crecip(b); }

template <typename To, typename From>
__host__ __device__ inline Cx<To> ccast(Cx<From> a) { return cx<To>((To)a.re, (To)a.im); }

template <typename R>
__host__ __device__ inline R cabs2(Cx<R> a) { return a.re * a.re + a.im * a.im; }

// One front of one panel of one problem (a node of the elimination tree).
struct FrontInst {
    int32_t s, u, start, wvoff;  // pivots, update size, first elimination position,
                                 // update-vector offset within the panel's class
    int32_t child0, child1;      // instance ids of the children, -1 if none
    int32_t uoff, moff;          // absolute offsets into the update-set and extend-add map arrays
    int32_t panel, depth;        // global panel id, depth in the tree
    int32_t cw0, cw1;            // update-vector offsets (wvoff) of the two children
    int64_t loff;                // offset of the (s+u) x s factor block (complex elements)
    int64_t woff;                // offset of the u x u update matrix in its depth-parity workspace
    int64_t doff;                // offset of the s reciprocal pivots
    int64_t toff;                // offset of the s x s block of L_F^{-1} in the scratch of its depth
    int32_t g0;                  // first column of G that is formed (a multiple of 64; see the inversion)
    int32_t pad;
};

// One workgroup of a forward or backward pass of a panel solve.  Offsets are
// relative to the panel (factors, pivots) or to the panel class (maps, pass
// vectors), except moff and pmap, which index the concatenated map arrays.
struct SolveItem {
    int64_t loff;            // the front's (s+u) x s block of G
    int32_t n, s, start;     // rows, pivots, first elimination position
    int32_t blk;             // first row (forward) or column (backward) of the workgroup
    int32_t moff;            // extend-add maps: 2n entries, position in child 0 / 1 update set or -1
    int32_t c2;              // the front's child-contribution slots (2n per right-hand side)
    int32_t push;            // forward: the front's slot in its parent's contributions, -1 at the root
    int32_t pmap;            // forward: position of each update entry in the parent front
    int32_t xu;              // the front's update-set values (u per right-hand side)
    int32_t cxu0, cxu1;      // backward: the children's update-set values, -1 if no child
    // the front's cells, a rectangle: (x0 | y0 << 16) and (cells per row |
    // cells << 16); pivot e is cell e mod cells (row-major) on aux plane e / cells
    int32_t cell0, cellw;
    int32_t leaf;            // 1 if the front has no children
};
static_assert(sizeof(SolveItem) == 64, "SolveItem is one 64-byte scalar load");

// Everything a pass kernel needs besides its work item; passed by value.
template <typename T>
struct PassArgs {
    const SolveItem* items;
    const Cx<T>* G;            // the panel's factors
    const Cx<T>* dinv;         // the panel's reciprocal pivots
    const int* cmap;           // extend-add maps (concatenated)
    const int* pmap;           // parent positions (concatenated)
    const int* hmap;           // matrix-core passes: parent pivot in h2 a first child adds into, or -1
    const Cx<double>* et;      // stretch tables
    const Cx<double>* src;     // forward: padded-grid input (column r at r * ld)
    Cx<double>* dst;           // backward: padded-grid output
    int64_t ld;
    Cx<T>* xmid;               // D^{-1} L^{-1} x in elimination order, column r at r * naux
    Cx<T>* c2;                 // child contributions, column r at r * c2ld
    Cx<T>* xu;                 // update-set values, column r at r * xuld
    int naux, c2ld, xuld, nrhs;
    int mode;                  // forward: 0 zero extension of the panel planes, 1 coupling
                               // J_{i+1,i}^T of the next plane; backward: 0 store, 1 subtract
    int couple;                // backward, mode 0: also subtract J_{i+1,i} x from the next plane
    int plane0;                // padded-grid plane held at offset 0 of src / dst
    int Nx, NxNy, nz, ga, lo, hi;
    int e1, e2, ie3hi;         // et offsets: e1 and e2 node tables, 1/e3 at the half plane below hi
    double inv_h2;
    // Matrix-core passes (groups of 16 right-hand sides): xu and c2 then
    // hold [entry][16] blocks, one block of entries per group, the group's
    // block of a buffer starting gs_* complex numbers after the previous one.
    // xu holds each front's [x_S; -x_U] (x_S from the forward pass in front
    // of the update-set values, which are stored negated; xmid is unused);
    // c2 is the panel class's own region (zero where no child writes) and h2
    // holds the right-hand side in elimination order (zero on the auxiliary
    // planes), written by the scatter at the start of a solve.
    Cx<T>* h2;
    const int* perm;           // elimination position -> box index of the panel class
    int64_t gs_u, gs_c2, gs_h2;
    // split contraction (forms that divide each item's contraction over
    // nsplit workgroups): partial 64 x 16 blocks, item-major, then group,
    // then split; a finishing launch sums them in split order
    Cx<T>* part;
    int nsplit;
    // GMRES with the convergence test on the device: while *run is 0 (every
    // right-hand side converged) the pass kernels return at once; NULL: always run
    const int* run;
};

struct PanelDev {
    int32_t prob, cls, Nx, Ny, nz, ga, lo, hi;
    int32_t perm_off;    // offset into the elimination-order arrays
    int32_t e3_off;      // offset of this panel's x3 stretch tables (node nz, inverse half nz+1)
    int32_t inst_base;   // instance id of the panel's front 0
    int32_t nfront;
};

struct ProbDev {
    int32_t n[3], N[3];
    int32_t gamma, pad;
    int64_t Npad;
    double h, omega, alpha;
    int32_t e_off[3];    // per axis: node stretch (N_j) then inverse half-node stretch (N_j + 1)
    int32_t pad2;
    const double* c;     // interior velocity, x1 fastest
};

}  // namespace hsw
