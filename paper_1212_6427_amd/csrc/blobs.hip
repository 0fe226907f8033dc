// Per-blob FP64 kernels of the ICM step (Sec. III.C): midpoint predictor
// (step 1), forces, slip correction and excess-momentum change (step 4), the
// inertial right-hand side of step 6, the momentum-conserving blob velocity
// update (step 8, Eq. (update_u)) and the position update (step 9).
#include "icm_internal.h"

namespace icm {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void raise_flag(unsigned int* flag, unsigned int bit) { atomicOr(flag, bit); }

// Step 1: q^{n+1/2} = q^n + dt/2 J^n v^n.
__global__ void k_predict(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    const double qh = b.q[t] + 0.5 * bp.dt * b.Jn[t];
    if (!isfinite(qh)) raise_flag(b.flag, 1u);
    b.qh[t] = qh;
}

// Positions folded into the box, q - L floor(q / L), for pair distances.
__global__ void k_wrap(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    const double L = bp.box[t % 3];
    b.qw[t] = b.qh[t] - L * floor(b.qh[t] / L);
}

// F = f_const - k (q - c): the one-body forces at q^{n+1/2}.
__global__ void k_forces_init(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    double f = b.fconst[t];
    if (bp.spring_k != 0.0) f -= bp.spring_k * (b.qh[t] - bp.spring_c[t % 3]);
    b.F[t] = f;
}

// F += WCA pair forces (Eq. (WCA), minimum image, unordered pairs) at
// q^{n+1/2}. Block (bx, by) takes blobs i of tile bx against blobs j of
// tile by: tile by's folded positions sit in LDS, so the minimum image of a
// difference in (-L, L) is one conditional shift per axis; partial sums are
// added to F atomically.
constexpr int kPairTile = 64;

__global__ void __launch_bounds__(kThreads) k_pairs(BlobParams bp, BlobBufs b) {
    __shared__ double tile[3][kPairTile];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * kPairTile;
    const int jl = j0 + threadIdx.x;
    if (threadIdx.x < kPairTile && jl < bp.nb) {
        tile[0][threadIdx.x] = b.qw[3 * jl];
        tile[1][threadIdx.x] = b.qw[3 * jl + 1];
        tile[2][threadIdx.x] = b.qw[3 * jl + 2];
    }
    __syncthreads();
    if (i >= bp.nb) return;
    const double qx = b.qw[3 * i], qy = b.qw[3 * i + 1], qz = b.qw[3 * i + 2];
    const double s2 = bp.wca_sigma * bp.wca_sigma;
    const double rc2 = 1.2599210498948732 * s2;  // (2^(1/6) sigma)^2
    const double Lx = bp.box[0], Ly = bp.box[1], Lz = bp.box[2];
    const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
    const int cnt = min(kPairTile, bp.nb - j0);
    double fx = 0, fy = 0, fz = 0;
    bool any = false;
    for (int jj = 0; jj < cnt; ++jj) {
        double dx = qx - tile[0][jj], dy = qy - tile[1][jj], dz = qz - tile[2][jj];
        dx = dx > hx ? dx - Lx : (dx < -hx ? dx + Lx : dx);
        dy = dy > hy ? dy - Ly : (dy < -hy ? dy + Ly : dy);
        dz = dz > hz ? dz - Lz : (dz < -hz ? dz + Lz : dz);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2 && j0 + jj != i) {
            const double sr2 = s2 / r2;
            const double sr6 = sr2 * sr2 * sr2;
            const double f = 24.0 * bp.wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;
            fx += f * dx;
            fy += f * dy;
            fz += f * dz;
            any = true;
        }
    }
    if (any) {
        atomicAdd(&b.F[3 * i], fx);
        atomicAdd(&b.F[3 * i + 1], fy);
        atomicAdd(&b.F[3 * i + 2], fz);
    }
}

// Step 4: du = [FULL] (J^{n+1/2} - J^n) v^n + [VISCOUS|FULL] (nu dt/2) c_lag;
// dp = m_e (u^n - J^{n+1/2} v~ - du).
__global__ void k_inertial_dp(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    double du = 0.0;
    if (bp.slip == 2) du += b.Jhvn[t] - b.Jn[t];
    if (bp.slip >= 1) du += 0.5 * (bp.eta / bp.rho) * bp.dt * b.lag[t];
    b.du[t] = du;
    b.dp[t] = b.me[t / 3] * (b.u[t] - b.Jhvt[t] - du);
}

// Step 6 right-hand side: dp - m_e J dv~.
__global__ void k_inertial_dp2(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    b.dp2[t] = b.dp[t] - b.me[t / 3] * b.g[t];
}

// Step 8: u^{n+1} = J (v~ + dv~) + du for blobs with m_e != 0.
__global__ void k_inertial_u(BlobParams bp, BlobBufs b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    if (b.me[t / 3] != 0.0) b.u[t] = b.Jhvt[t] + b.g[t] + b.du[t];
}

// Step 9: q^{n+1} = q^n + dt/2 J^{n+1/2} (v^{n+1} + v^n); blobs with m_e = 0
// take u^{n+1} = J^{n+1/2} v^{n+1}. Raises the numeric flag on NaN/Inf or a
// displacement above h.
__global__ void k_final(BlobParams bp, BlobBufs b, double h) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * bp.nb) return;
    const double dq = 0.5 * bp.dt * (b.Jhvnew[t] + b.Jhvn[t]);
    const double qn = b.q[t] + dq;
    if (!isfinite(qn)) raise_flag(b.flag, 1u);
    if (fabs(dq) > h) raise_flag(b.flag, 2u);
    b.q[t] = qn;
    if (b.me[t / 3] == 0.0) b.u[t] = b.Jhvnew[t];
}

__global__ void k_blob_diag(int nb, const double* me, const double* u, double* acc) {
    // single block: sum m_e u (3) and sum m_e u^2 / 2
    __shared__ double red[4][kThreads];
    double s[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        const double m = me[i];
        s[0] += m * u[3 * i];
        s[1] += m * u[3 * i + 1];
        s[2] += m * u[3 * i + 2];
        s[3] += 0.5 * m * (u[3 * i] * u[3 * i] + u[3 * i + 1] * u[3 * i + 1] + u[3 * i + 2] * u[3 * i + 2]);
    }
    for (int m = 0; m < 4; ++m) red[m][threadIdx.x] = s[m];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int m = 0; m < 4; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int m = 0; m < 4; ++m) acc[m] = red[m][0];
}

dim3 grid3(int nb) { return dim3((unsigned)((3 * nb + kThreads - 1) / kThreads)); }

}  // namespace

void launch_predict(const BlobParams& bp, const BlobBufs& b, hipStream_t s) {
    if (bp.nb > 0) hipLaunchKernelGGL(k_predict, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
}
void launch_forces(const BlobParams& bp, const BlobBufs& b, hipStream_t s) {
    if (bp.nb <= 0) return;
    hipLaunchKernelGGL(k_forces_init, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
    if (bp.wca_eps != 0.0 && bp.nb > 1) {
        hipLaunchKernelGGL(k_wrap, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
        const unsigned ti = (unsigned)((bp.nb + kThreads - 1) / kThreads);
        const unsigned tj = (unsigned)((bp.nb + kPairTile - 1) / kPairTile);
        hipLaunchKernelGGL(k_pairs, dim3(ti, tj), dim3(kThreads), 0, s, bp, b);
    }
}
void launch_inertial_dp(const BlobParams& bp, const BlobBufs& b, hipStream_t s) {
    if (bp.nb > 0) hipLaunchKernelGGL(k_inertial_dp, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
}
void launch_inertial_dp2(const BlobParams& bp, const BlobBufs& b, hipStream_t s) {
    if (bp.nb > 0) hipLaunchKernelGGL(k_inertial_dp2, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
}
void launch_inertial_u(const BlobParams& bp, const BlobBufs& b, hipStream_t s) {
    if (bp.nb > 0) hipLaunchKernelGGL(k_inertial_u, grid3(bp.nb), dim3(kThreads), 0, s, bp, b);
}
void launch_final(const BlobParams& bp, const BlobBufs& b, double h, hipStream_t s) {
    if (bp.nb > 0) hipLaunchKernelGGL(k_final, grid3(bp.nb), dim3(kThreads), 0, s, bp, b, h);
}
void launch_blob_diag(int nb, const double* me, const double* u, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_blob_diag, dim3(1), dim3(kThreads), 0, s, nb, me, u, acc);
}

}  // namespace icm
