// Grid kernels of the ICM step: the right-hand side of the unperturbed fluid
// solve (step 2 of Sec. III.C) with the staggered stochastic stress of
// Sec. III.B.2, spreading S and interpolation J of Sec. III.A.1, the
// equilibrium initial sample, and FP64 field reductions.
#include "icm_internal.h"

namespace icm {

namespace {

constexpr int kThreads = 256;

template <typename T>
struct NormalPair {
    T a, b;
};

template <typename T>
__device__ __forceinline__ NormalPair<T> bm(uint32_t wa, uint32_t wb) {
    NormalPair<T> r;
    box_muller(wa, wb, r.a, r.b);
    return r;
}

// Right-hand side of the unperturbed solve (Eq. (provisional_step-1)):
//   rhs_a = (rho/dt) v_a + (eta/2) (L v)_a + s (D_w Sigma-hat)_a + f_body,a
// with Sigma-hat = W + W^T realised as 2 W_aa at cell centres and
// sqrt(2) W_ab on edges. One thread per cell; the neighbouring cells' normals
// are regenerated from their Philox counters.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rhs(GridDesc<T> g, RhsCoef c) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int i = (int)(cell % nx);
    const int j = (int)((cell / nx) % ny);
    const int k = (int)(cell / ((long long)nx * ny));
    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
    const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
    auto lin = [&](int a, int b, int d) -> long long { return ((long long)d * ny + b) * nx + a; };
    const long long cip = lin(ip, j, k), cim = lin(im, j, k);
    const long long cjp = lin(i, jp, k), cjm = lin(i, jm, k);
    const long long ckp = lin(i, j, kp), ckm = lin(i, j, km);
    T out[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T* v = g.v + a * g.ncell;
        const T v0 = v[cell];
        const T lap = v[cip] + v[cim] + v[cjp] + v[cjm] + v[ckp] + v[ckm] - (T)6 * v0;
        out[a] = (T)c.rho_dt * v0 + (T)c.half_eta_h2 * lap + (T)c.body[a];
    }
    if (c.noise != 0.0) {
        const NoiseKey& nk = c.key;
        // own cell: block 0 -> (xx, yy), (zz, xy); block 1 -> (xz, yz)
        const u32x4 o0 = noise_words(nk, (uint32_t)cell, 0);
        const u32x4 o1 = noise_words(nk, (uint32_t)cell, 1);
        const NormalPair<T> oxy = bm<T>(o0.x, o0.y);   // xx, yy
        const NormalPair<T> ozx = bm<T>(o0.z, o0.w);   // zz, xy
        const NormalPair<T> oxz = bm<T>(o1.x, o1.y);   // xz, yz
        const T wxx = oxy.a, wyy = oxy.b, wzz = ozx.a, wxy = ozx.b, wxz = oxz.a, wyz = oxz.b;
        // neighbours
        const u32x4 nim = noise_words(nk, (uint32_t)cim, 0);
        const T wxx_im = bm<T>(nim.x, nim.y).a;
        const u32x4 nip0 = noise_words(nk, (uint32_t)cip, 0);
        const u32x4 nip1 = noise_words(nk, (uint32_t)cip, 1);
        const T wxy_ip = bm<T>(nip0.z, nip0.w).b;
        const T wxz_ip = bm<T>(nip1.x, nip1.y).a;
        const u32x4 njm = noise_words(nk, (uint32_t)cjm, 0);
        const T wyy_jm = bm<T>(njm.x, njm.y).b;
        const u32x4 njp0 = noise_words(nk, (uint32_t)cjp, 0);
        const u32x4 njp1 = noise_words(nk, (uint32_t)cjp, 1);
        const T wxy_jp = bm<T>(njp0.z, njp0.w).b;
        const T wyz_jp = bm<T>(njp1.x, njp1.y).b;
        const u32x4 nkm = noise_words(nk, (uint32_t)ckm, 0);
        const T wzz_km = bm<T>(nkm.z, nkm.w).a;
        const u32x4 nkp = noise_words(nk, (uint32_t)ckp, 1);
        const NormalPair<T> kxz = bm<T>(nkp.x, nkp.y);
        const T wxz_kp = kxz.a, wyz_kp = kxz.b;
        const T r2 = (T)1.41421356237309504880;
        const T dx = (T)2 * (wxx - wxx_im) + r2 * (wxy_jp - wxy) + r2 * (wxz_kp - wxz);
        const T dy = r2 * (wxy_ip - wxy) + (T)2 * (wyy - wyy_jm) + r2 * (wyz_kp - wyz);
        const T dz = r2 * (wxz_ip - wxz) + r2 * (wyz_jp - wyz) + (T)2 * (wzz - wzz_km);
        const T s = (T)c.noise;
        out[0] += s * dx;
        out[1] += s * dy;
        out[2] += s * dz;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) g.rhs[a * g.ncell + cell] = out[a];
}

// Equilibrium sample: every face N(0, sd^2) from Philox block 2 of the cell
// (words (w0,w1) -> (x, y) faces, (w2,w3) -> (z face, unused)).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_eq_noise(GridDesc<T> g, double sd, NoiseKey nk) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const u32x4 w = noise_words(nk, (uint32_t)cell, 2);
    double a, b, cz, unused;
    box_muller(w.x, w.y, a, b);
    box_muller(w.z, w.w, cz, unused);
    g.rhs[cell] = (T)(sd * a);
    g.rhs[g.ncell + cell] = (T)(sd * b);
    g.rhs[2 * g.ncell + cell] = (T)(sd * cz);
}

template <typename T>
__global__ void k_zero(T* p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

template <typename T>
__global__ void k_axpy(T* y, const T* x, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] += x[i];
}

// Component grid origin along axis beta for component a: 0 if beta == a
// (faces normal to a), else 1/2 (cell centres).
__device__ __forceinline__ double comp_offset(int beta, int a) { return beta == a ? 0.0 : 0.5; }

// S: field_a += h^-3 phi(dx) phi(dy) phi(dz) val_a. One thread per
// (blob, component); atomics resolve overlapping kernels.
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_spread(GridDesc<T> g, T* field, int nb, const double* __restrict__ q,
                                                    const double* __restrict__ F, const double* __restrict__ coef,
                                                    int deriv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / 3, a = t - 3 * (t / 3);
    if (b >= nb) return;
    const double inv_h = 1.0 / g.h;
    double val = (F ? F[3 * b + a] : 1.0) * (coef ? coef[b] : 1.0) * inv_h * inv_h * inv_h;
    AxisStencil<P> sx, sy, sz;
    axis_stencil<P>(q[3 * b + 0] * inv_h - comp_offset(0, a), g.nx, deriv && a == 0, inv_h, sx);
    axis_stencil<P>(q[3 * b + 1] * inv_h - comp_offset(1, a), g.ny, deriv && a == 1, inv_h, sy);
    axis_stencil<P>(q[3 * b + 2] * inv_h - comp_offset(2, a), g.nz, deriv && a == 2, inv_h, sz);
    T* f = field + a * g.ncell;
    for (int c = 0; c < P; ++c) {
        for (int bb = 0; bb < P; ++bb) {
            const double wzy = sz.w[c] * sy.w[bb] * val;
            const long long row = ((long long)sz.node[c] * g.ny + sy.node[bb]) * g.nx;
#pragma unroll
            for (int aa = 0; aa < P; ++aa) atomicAdd(&f[row + sx.node[aa]], (T)(wzy * sx.w[aa]));
        }
    }
}

// J: out[b][a] = sum phi(dx) phi(dy) phi(dz) f_a (FP64 accumulation); with
// lap = 1 the field value at each node is replaced by its 7-point Laplacian.
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_gather(GridDesc<T> g, const T* __restrict__ field, int nb,
                                                    const double* __restrict__ q, double* __restrict__ out, int lap) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / 3, a = t - 3 * (t / 3);
    if (b >= nb) return;
    const double inv_h = 1.0 / g.h;
    AxisStencil<P> sx, sy, sz;
    axis_stencil<P>(q[3 * b + 0] * inv_h - comp_offset(0, a), g.nx, false, inv_h, sx);
    axis_stencil<P>(q[3 * b + 1] * inv_h - comp_offset(1, a), g.ny, false, inv_h, sy);
    axis_stencil<P>(q[3 * b + 2] * inv_h - comp_offset(2, a), g.nz, false, inv_h, sz);
    const T* f = field + a * g.ncell;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    double acc = 0.0;
    for (int c = 0; c < P; ++c) {
        for (int bb = 0; bb < P; ++bb) {
            const double wzy = sz.w[c] * sy.w[bb];
            const int k = sz.node[c], j = sy.node[bb];
            const long long row = ((long long)k * ny + j) * nx;
#pragma unroll
            for (int aa = 0; aa < P; ++aa) {
                const int i = sx.node[aa];
                double val;
                if (!lap) {
                    val = (double)f[row + i];
                } else {
                    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
                    const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
                    const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
                    const double c0 = (double)f[row + i];
                    val = ((double)f[row + ip] + (double)f[row + im] +
                           (double)f[((long long)k * ny + jp) * nx + i] + (double)f[((long long)k * ny + jm) * nx + i] +
                           (double)f[((long long)kp * ny + j) * nx + i] + (double)f[((long long)km * ny + j) * nx + i] -
                           6.0 * c0) * inv_h * inv_h;
                }
                acc += wzy * sx.w[aa] * val;
            }
        }
    }
    out[3 * b + a] = acc;
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// FP64 field diagnostics: momentum, kinetic energy, max |v|, max |D v|.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_field_diag(GridDesc<T> g, double rho, double* acc) {
    __shared__ double red[5][kThreads / 64];
    double s0 = 0, s1 = 0, s2 = 0, ke = 0, vmax = 0, dmax = 0;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncell;
         cell += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(cell % nx);
        const int j = (int)((cell / nx) % ny);
        const int k = (int)(cell / ((long long)nx * ny));
        const double vx = g.v[cell], vy = g.v[g.ncell + cell], vz = g.v[2 * g.ncell + cell];
        s0 += vx;
        s1 += vy;
        s2 += vz;
        ke += vx * vx + vy * vy + vz * vz;
        vmax = fmax(vmax, fmax(fabs(vx), fmax(fabs(vy), fabs(vz))));
        const long long cip = ((long long)k * ny + j) * nx + (i + 1 == nx ? 0 : i + 1);
        const long long cjp = ((long long)k * ny + (j + 1 == ny ? 0 : j + 1)) * nx + i;
        const long long ckp = ((long long)(k + 1 == nz ? 0 : k + 1) * ny + j) * nx + i;
        const double div = ((double)g.v[cip] - vx) + ((double)g.v[g.ncell + cjp] - vy) +
                           ((double)g.v[2 * g.ncell + ckp] - vz);
        dmax = fmax(dmax, fabs(div));
    }
    double vals[5] = {s0, s1, s2, ke, 0};
    for (int off = 32; off > 0; off >>= 1) {
        for (int m = 0; m < 4; ++m) vals[m] += __shfl_down(vals[m], off);
        vmax = fmax(vmax, __shfl_down(vmax, off));
        dmax = fmax(dmax, __shfl_down(dmax, off));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        for (int m = 0; m < 4; ++m) red[m][wv] = vals[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double cv = g.h * g.h * g.h * rho;
        double t[4] = {0, 0, 0, 0};
        for (int w = 0; w < kThreads / 64; ++w)
            for (int m = 0; m < 4; ++m) t[m] += red[m][w];
        atomicAdd(&acc[0], cv * t[0]);
        atomicAdd(&acc[1], cv * t[1]);
        atomicAdd(&acc[2], cv * t[2]);
        atomicAdd(&acc[3], 0.5 * cv * t[3]);
    }
    if (lane == 0) {
        atomic_max_nonneg(&acc[4], vmax);
        atomic_max_nonneg(&acc[5], dmax);
    }
}

unsigned grid_for(long long n) {
    long long b = (n + kThreads - 1) / kThreads;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

template <typename T>
void launch_rhs(const GridDesc<T>& g, const RhsCoef& c, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs<T>, dim3(grid_for(g.ncell)), dim3(kThreads), 0, s, g, c);
}

template <typename T>
void launch_equilibrium_noise(const GridDesc<T>& g, double sd, NoiseKey key, hipStream_t s) {
    hipLaunchKernelGGL(k_eq_noise<T>, dim3(grid_for(g.ncell)), dim3(kThreads), 0, s, g, sd, key);
}

template <typename T>
void launch_zero(T* p, long long n, hipStream_t s) {
    long long b = (n + kThreads - 1) / kThreads;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)b), dim3(kThreads), 0, s, p, n);
}

template <typename T>
void launch_axpy(T* y, const T* x, long long n, hipStream_t s) {
    long long b = (n + kThreads - 1) / kThreads;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_axpy<T>, dim3((unsigned)b), dim3(kThreads), 0, s, y, x, n);
}

template <typename T>
void launch_spread(const GridDesc<T>& g, T* field, int kernel, int nb, const double* q, const double* F,
                   const double* coef, bool deriv, hipStream_t s) {
    if (nb <= 0) return;
    const dim3 grid(grid_for(3LL * nb));
    if (kernel == 3)
        hipLaunchKernelGGL((k_spread<T, 3>), grid, dim3(kThreads), 0, s, g, field, nb, q, F, coef, deriv ? 1 : 0);
    else
        hipLaunchKernelGGL((k_spread<T, 4>), grid, dim3(kThreads), 0, s, g, field, nb, q, F, coef, deriv ? 1 : 0);
}

template <typename T>
void launch_gather(const GridDesc<T>& g, const T* field, int kernel, int nb, const double* q, double* out,
                   bool laplacian, hipStream_t s) {
    if (nb <= 0) return;
    const dim3 grid(grid_for(3LL * nb));
    if (kernel == 3)
        hipLaunchKernelGGL((k_gather<T, 3>), grid, dim3(kThreads), 0, s, g, field, nb, q, out, laplacian ? 1 : 0);
    else
        hipLaunchKernelGGL((k_gather<T, 4>), grid, dim3(kThreads), 0, s, g, field, nb, q, out, laplacian ? 1 : 0);
}

template <typename T>
void launch_field_diag(const GridDesc<T>& g, double rho, double* acc, hipStream_t s) {
    long long b = (g.ncell + kThreads - 1) / kThreads;
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(k_field_diag<T>, dim3((unsigned)b), dim3(kThreads), 0, s, g, rho, acc);
}

#define ICM_INST(T)                                                                                        \
    template void launch_rhs<T>(const GridDesc<T>&, const RhsCoef&, hipStream_t);                         \
    template void launch_equilibrium_noise<T>(const GridDesc<T>&, double, NoiseKey, hipStream_t);         \
    template void launch_zero<T>(T*, long long, hipStream_t);                                              \
    template void launch_axpy<T>(T*, const T*, long long, hipStream_t);                                    \
    template void launch_spread<T>(const GridDesc<T>&, T*, int, int, const double*, const double*,        \
                                   const double*, bool, hipStream_t);                                     \
    template void launch_gather<T>(const GridDesc<T>&, const T*, int, int, const double*, double*, bool, \
                                   hipStream_t);                                                          \
    template void launch_field_diag<T>(const GridDesc<T>&, double, double*, hipStream_t);
ICM_INST(float)
ICM_INST(double)
#undef ICM_INST

}  // namespace icm
