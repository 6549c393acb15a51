// Assembly inputs: velocity checks and the 1D complex-stretch tables from
// which every entry of A and of the auxiliary problems H_i is generated.
//
// PML (Sec. 1.1: a radiation condition represented by PML; the amplitude C is
// the one the experiments tune, Sec. 3): at depth t past the last interior
// node, sigma(t) = (C/eta)(t/eta)^2 with eta = (gamma + 1) h (the Dirichlet
// wall), and the stretch is e = 1 + i sigma(t)/omega, which damps outgoing
// waves e^{+ikx} under the e^{-i omega t} convention of Sec. 1.  For panel i
// >= 1 the x3 stretch of the gamma planes prefixed to the panel, and of the
// half-planes up to the panel, is the artificial profile with depth measured
// from the panel's first plane (Sec. 1.1, Alg. 1.4: "prefixing PML").
#include "devtypes.hpp"
#include "kernels.hpp"

namespace hsw {

__device__ inline Cx<double> stretch_at(double t, double C, double eta, double omega) {
    const double sg = (C / eta) * (t / eta) * (t / eta);
    return cx<double>(1.0, sg / omega);
}

__device__ inline double phys_depth(double x, int nj, double h) {
    return fmax(0.0, fmax(h - x, x - nj * h));
}

// Physical table of one axis: node stretch (N entries) then inverse half-node
// stretch (N+1 entries, entry a between nodes a-1 and a).
__global__ void k_axis_table(Cx<double>* __restrict__ out, int nj, int gj, double h, double C,
                             double omega) {
    const int N = nj + 2 * gj;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a > 2 * N) return;
    const bool node = a < N;
    const int ia = node ? a : a - N;
    const double x = (ia - gj + 1) * h - (node ? 0.0 : 0.5 * h);
    Cx<double> e = cx<double>(1.0, 0.0);
    if (gj > 0 && C != 0.0) e = stretch_at(phys_depth(x, nj, h), C, (gj + 1) * h, omega);
    out[a] = node ? e : crecip(e);
}

// x3 table of a panel's auxiliary box: nz node stretches then nz+1 inverse
// half-node stretches; ga artificial planes precede the panel planes [lo, hi).
__global__ void k_aux_table(Cx<double>* __restrict__ out, int n3, int g, int lo, int ga, int nz,
                            double h, double C, double omega) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a > 2 * nz) return;
    const bool node = a < nz;
    const int ia = node ? a : a - nz;
    const double eta = (g + 1) * h;
    double t;
    if (node) {
        t = ia < ga ? (ga - ia) * h : phys_depth((lo - ga + ia - g + 1) * h, n3, h);
    } else {
        t = (ga > 0 && ia <= ga) ? (ga - ia + 0.5) * h
                                 : phys_depth((lo - ga + ia - g + 1) * h - 0.5 * h, n3, h);
    }
    Cx<double> e = cx<double>(1.0, 0.0);
    if (g > 0 && C != 0.0) e = stretch_at(t, C, eta, omega);
    out[a] = node ? e : crecip(e);
}

// bad[0] = 1 if any velocity is not positive and finite.
__global__ void k_check_velocity(const double* __restrict__ c, int64_t n, int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double v = c[i];
    if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
}

void launch_axis_table(Cx<double>* out, int nj, int gj, double h, double C, double omega,
                       hipStream_t st) {
    const int cnt = 2 * (nj + 2 * gj) + 1;
    hipLaunchKernelGGL(k_axis_table, dim3((cnt + 255) / 256), dim3(256), 0, st, out, nj, gj, h, C, omega);
}
void launch_aux_table(Cx<double>* out, int n3, int g, int lo, int ga, int nz, double h, double C,
                      double omega, hipStream_t st) {
    const int cnt = 2 * nz + 1;
    hipLaunchKernelGGL(k_aux_table, dim3((cnt + 255) / 256), dim3(256), 0, st, out, n3, g, lo, ga, nz, h,
                       C, omega);
}
void launch_check_velocity(const double* c, int64_t n, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_check_velocity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c, n, bad);
}

}  // namespace hsw
