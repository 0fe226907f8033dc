// Per-blob FP64 kernels of the ICM step (Sec. III.C): forces at the
// midpoint, slip correction and excess-momentum change (step 4), the inertial
// right-hand side of step 6 and the momentum-conserving blob velocity update
// (step 8, Eq. (update_u)). The predictor (step 1) and the position update
// (step 9) are fused with their gathers in grid.hip.
#include "icm_internal.h"

namespace icm {

namespace {

constexpr int kThreads = 256;
constexpr int kTabThreads = 1024;  // the projection-table kernel: one workgroup per replica


// F += WCA pair forces (Eq. (WCA), minimum image, unordered pairs counted
// once) at q^{n+1/2}: each blob walks the lists of the 27 cells around its
// own (cells are at least one cutoff wide, at least 3 per axis). Replica
// blockIdx.y.
// Workgroups from pair_blocks on bin the replica's blobs for the RHS spread
// instead (any pair mode; width: the stencil width), which needs only the
// stencil records of the step-1 gather, like the pair walk its positions.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_pairs_cells(const RepDesc<T>* __restrict__ rd, int pair_blocks,
                                                          int width) {
    if ((int)blockIdx.x >= pair_blocks) {
        const int b = ((int)blockIdx.x - pair_blocks) * (int)blockDim.x + (int)threadIdx.x;
        if (width == 3)
            bin_blob_from_records<T, 3>(rd[blockIdx.y], b);
        else
            bin_blob_from_records<T, 4>(rd[blockIdx.y], b);
        return;
    }
    if (rd[blockIdx.y].pair_mode != 1) return;
    const BlobParams bp = rd[blockIdx.y].bp;
    const BlobBufs b = rd[blockIdx.y].bb;
    const CellGrid cg = rd[blockIdx.y].cg;
    const unsigned long long stamp = cell_stamp(*rd[blockIdx.y].step);
    // four lanes per blob, each walking every fourth of the 27 cells
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t >> 2, sub = t & 3;
    const bool active = i < bp.nb;
    double fx = 0, fy = 0, fz = 0;
    if (active) {
        const double qx = b.qw[3 * i], qy = b.qw[3 * i + 1], qz = b.qw[3 * i + 2];
        const double s2 = bp.wca_sigma * bp.wca_sigma;
        const double rc2 = 1.2599210498948732 * s2;  // (2^(1/6) sigma)^2
        const double Lx = bp.box[0], Ly = bp.box[1], Lz = bp.box[2];
        const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
        const double q3[3] = {qx, qy, qz};
        // neighbour cell coordinates per axis, wrapped (n >= 3)
        int lo[3], mid[3], hi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int cc = (int)(q3[a] * cg.inv_size[a]);
            mid[a] = cc >= cg.n[a] ? cg.n[a] - 1 : (cc < 0 ? 0 : cc);
            lo[a] = mid[a] == 0 ? cg.n[a] - 1 : mid[a] - 1;
            hi[a] = mid[a] + 1 == cg.n[a] ? 0 : mid[a] + 1;
        }
        auto pick = [](const int* l, const int* m, const int* h, int a, int d) {
            return d == 0 ? l[a] : (d == 1 ? m[a] : h[a]);
        };
        // this lane's (up to 7) head loads are independent: issue them first
        const gptr<const unsigned long long> heads = as_global((const unsigned long long*)cg.heads);
        unsigned long long hv[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int n = sub + 4 * m;
            hv[m] = 0;
            if (n < 27) {
                const int z = pick(lo, mid, hi, 2, n / 9), y = pick(lo, mid, hi, 1, (n / 3) % 3);
                const int x = pick(lo, mid, hi, 0, n % 3);
                hv[m] = heads[((long long)z * cg.n[1] + y) * cg.n[0] + x];
            }
        }
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            if (sub + 4 * m >= 27) break;
            const unsigned long long h = hv[m];
            int j = ((h >> kHeadBlobBits) == stamp) ? (int)(h & ((1u << kHeadBlobBits) - 1)) : -1;
            while (j >= 0) {
                if (j != i) {
                    double ex = qx - b.qw[3 * j], ey = qy - b.qw[3 * j + 1], ez = qz - b.qw[3 * j + 2];
                    ex = ex > hx ? ex - Lx : (ex < -hx ? ex + Lx : ex);
                    ey = ey > hy ? ey - Ly : (ey < -hy ? ey + Ly : ey);
                    ez = ez > hz ? ez - Lz : (ez < -hz ? ez + Lz : ez);
                    const double r2 = ex * ex + ey * ey + ez * ez;
                    if (r2 < rc2 && r2 > 0.0) {
                        const double sr2 = s2 / r2;
                        const double sr6 = sr2 * sr2 * sr2;
                        const double f = 24.0 * bp.wca_eps * (2.0 * sr6 * sr6 - sr6) / r2;
                        fx += f * ex;
                        fy += f * ey;
                        fz += f * ez;
                    }
                }
                j = cg.next[j];
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 4; off <<= 1) {
        fx += __shfl_xor(fx, off, 4);
        fy += __shfl_xor(fy, off, 4);
        fz += __shfl_xor(fz, off, 4);
    }
    if (active && sub == 0) {
        b.F[3 * i] += fx;
        b.F[3 * i + 1] += fy;
        b.F[3 * i + 2] += fz;
    }
}

// All-pairs WCA forces, for boxes too small for a 3-cell list: block (bx, by)
// takes blobs i of tile bx against the folded positions of the kPairTile blobs
// of tile by held in LDS; partial sums are added to F atomically. Replica
// blockIdx.z.
constexpr int kPairTile = 64;

template <typename T>
__global__ void __launch_bounds__(kThreads) k_pairs(const RepDesc<T>* __restrict__ rd) {
    __shared__ double tile[3][kPairTile];
    if (rd[blockIdx.z].pair_mode != 2) return;
    const BlobParams bp = rd[blockIdx.z].bp;
    const BlobBufs b = rd[blockIdx.z].bb;
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

// With the mean velocity carried in FP64: the sum over a replica's blobs of
// the step-6 source dp - m_e g, formed again here in a fixed order (one
// workgroup per replica).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_dp2_sum(const RepDesc<T>* __restrict__ rd) {
    const BlobBufs b = rd[blockIdx.x].bb;
    block_sum3<true>(rd[blockIdx.x].bp.nb, b.dp, b.me, b.g, rd[blockIdx.x].g.k0 + 6);
}

// Step 5 for replicas with at most kTabMaxBlobs blobs: g_i = J_i dv~ with
// dv~ = P S (c5 dp). Since dv~ enters the step only through J, it is never
// formed: with K the tabulated real-space kernel of the discrete
// projection, g_i,a = sum_j sum_b sum_{nodes x of J_i,a, y of S_j,b}
// w(x) w(y) h^-3 K_ab[x - y] c5_j dp_j,b, the same linear map as spreading,
// projecting and interpolating. The node weights are products over the
// axes, so the double sum over nodes is a sum over the (2P - 1)^3 offsets s
// of K_ab[base_i - base_j + s] times the product of the three 1-D
// correlations c(s) = sum_m w_i[m] w_j[m - s] of the two stencils' weights.
// One workgroup per replica; each output is summed in a fixed order. Then
// the step-6 source dp2 = dp - m_e g, u^{n+1} = J v~ + g + du for m_e != 0
// (step 8) and, with the mean velocity carried in FP64, the sum of dp2.
template <int P>
__device__ __forceinline__ double stencil_corr(const double* wa, const double* wb, int s) {
    double c = 0.0;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int n = m - s;
        if (n >= 0 && n < P) c += wa[m] * wb[n];
    }
    return c;
}

__device__ __forceinline__ int wrap_offset(int d, int n) {
    d %= n;
    return d < 0 ? d + n : d;
}

// The replica's stencil records and sources are staged in LDS first, so that
// each item's only global reads are the Q table values of its x-row.
template <typename T, int P>
__global__ void __launch_bounds__(kTabThreads) k_jps_table(const RepDesc<T>* __restrict__ rd) {
    constexpr int Q = 2 * P - 1;
    constexpr int kWaves = kTabThreads / 64;
    __shared__ double s_rec[3 * kTabMaxBlobs * kStcPerComp];
    __shared__ double s_f[3 * kTabMaxBlobs];
    __shared__ double s_g[3 * kTabMaxBlobs];
    __shared__ double s_part[3 * kTabMaxBlobs][kWaves];
    const GridDesc<T>& g = rd[blockIdx.x].g;
    const BlobBufs& b = rd[blockIdx.x].bb;
    const int nb = rd[blockIdx.x].bp.nb;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long long ncell = g.ncell;
    const double ih3 = 1.0 / (g.h * g.h * g.h);
    const gptr<const T> K = as_global(g.ptab);
    for (int t = threadIdx.x; t < 3 * nb * kStcPerComp; t += blockDim.x) s_rec[t] = b.stc[t];
    for (int t = threadIdx.x; t < 3 * nb; t += blockDim.x) s_f[t] = b.c5[t / 3] * b.dp[t] * ih3;
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    // W waves per output (i, a) (several when there are fewer outputs than
    // waves); their lanes take the items (j, b, z offset, y offset), the x
    // offsets run inside an item
    const int nout = 3 * nb;
    const int W = (nout > 0 && nout < kWaves) ? kWaves / nout : 1;
    const int ws = wave % W;
    for (int o = wave / W; o < nout && wave < W * nout; o += kWaves / W) {
        const int al = o - 3 * (o / 3);
        const double* oi = s_rec + o * kStcPerComp;
        double part = 0.0;
        for (int it = lane + 64 * ws; it < nb * 3 * Q * Q; it += 64 * W) {
            const int jb = it / (Q * Q), rem = it - jb * Q * Q;  // jb = 3 j + b
            const int tz = rem / Q, ty = rem - tz * Q;
            const double fj = s_f[jb];
            if (fj == 0.0) continue;
            const double* oj = s_rec + jb * kStcPerComp;
            const double cyz = stencil_corr<P>(oi + 11, oj + 11, tz - (P - 1)) * stencil_corr<P>(oi + 7, oj + 7, ty - (P - 1));
            if (cyz == 0.0) continue;
            const int be = jb - 3 * (jb / 3);
            const int dz = wrap_offset((int)oi[2] - (int)oj[2] + tz - (P - 1), nz);
            const int dy = wrap_offset((int)oi[1] - (int)oj[1] + ty - (P - 1), ny);
            const gptr<const T> row = K + (long long)(be * 3 + al) * ncell + ((long long)dz * ny + dy) * nx;
            const int dx0 = wrap_offset((int)oi[0] - (int)oj[0] - (P - 1), nx);
            T kv[Q];
#pragma unroll
            for (int tx = 0; tx < Q; ++tx) {
                // dx0 + tx < nx + 2P - 2 <= 3 nx: an axis narrower than the
                // 2P - 1 offsets (four nodes with P = 4) wraps twice
                int x = dx0 + tx;
                if (x >= nx) x -= nx;
                if (x >= nx) x -= nx;
                kv[tx] = row[x];
            }
            double sx = 0.0;
#pragma unroll
            for (int tx = 0; tx < Q; ++tx) sx += stencil_corr<P>(oi + 3, oj + 3, tx - (P - 1)) * (double)kv[tx];
            part += fj * cyz * sx;
        }
        // butterfly sum over the wave, then over the output's W waves in
        // order (the same order on every run)
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (lane == 0) s_part[o][ws] = part;
    }
    __syncthreads();
    if ((int)threadIdx.x < nout) {
        const int o = (int)threadIdx.x;
        double sum = 0.0;
        for (int k = 0; k < W; ++k) sum += s_part[o][k];
        s_g[o] = sum;
        b.g[o] = sum;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * nb; t += blockDim.x) {
        const double me = b.me[t / 3], gt = s_g[t];
        b.dp2[t] = b.dp[t] - me * gt;
        if (me != 0.0) b.u[t] = b.Jhvt[t] + gt + b.du[t];
    }
    if (g.k0) block_sum3<true>(nb, b.dp, b.me, s_g, g.k0 + 6);
}

__global__ void k_blob_diag(int nb, const double* me, const double* u, double* acc) {
    // single block: sum m_e u (3), sum m_e u^2 / 2, and the largest velocity
    // component max |u_a| (for the advective CFL number)
    __shared__ double red[5][kThreads];
    double s[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        const double m = me[i];
        const double ux = u[3 * i], uy = u[3 * i + 1], uz = u[3 * i + 2];
        s[0] += m * ux;
        s[1] += m * uy;
        s[2] += m * uz;
        s[3] += 0.5 * m * (ux * ux + uy * uy + uz * uz);
        s[4] = fmax(s[4], fmax(fabs(ux), fmax(fabs(uy), fabs(uz))));
    }
    for (int m = 0; m < 5; ++m) red[m][threadIdx.x] = s[m];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int m = 0; m < 4; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + off];
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int m = 0; m < 5; ++m) acc[m] = red[m][0];
}

}  // namespace

template <typename T>
void launch_forces(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb <= 0) return;
    // the one-body forces, the cell lists and the stencil records are set by
    // the gathers before; the cell-list pair walk and the RHS bins share a
    // launch (the bins get workgroups of their own), else the bins run alone
    if (B.any_cells) {
        const unsigned pair_blocks = (unsigned)((4LL * B.max_nb + kThreads - 1) / kThreads);
        const unsigned bin_blocks = (unsigned)((B.max_nb + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_pairs_cells<T>, dim3(pair_blocks + bin_blocks, B.nrep), dim3(kThreads), 0, s, B.d,
                           (int)pair_blocks, B.kernel);
    } else {
        launch_bins(B, s);
    }
    if (B.any_all_pairs) {
        const unsigned ti = (unsigned)((B.max_nb + kThreads - 1) / kThreads);
        const unsigned tj = (unsigned)((B.max_nb + kPairTile - 1) / kPairTile);
        hipLaunchKernelGGL(k_pairs<T>, dim3(ti, tj, B.nrep), dim3(kThreads), 0, s, B.d);
    }
}
template <typename T>
void launch_dp2_sum(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb > 0 && B.g.k0) hipLaunchKernelGGL(k_dp2_sum<T>, dim3(B.nrep), dim3(kThreads), 0, s, B.d);
}
template <typename T>
void launch_jps_table(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb <= 0) return;
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_jps_table<T, 3>), dim3(B.nrep), dim3(kTabThreads), 0, s, B.d);
    else
        hipLaunchKernelGGL((k_jps_table<T, 4>), dim3(B.nrep), dim3(kTabThreads), 0, s, B.d);
}
void launch_blob_diag(int nb, const double* me, const double* u, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_blob_diag, dim3(1), dim3(kThreads), 0, s, nb, me, u, acc);
}

#define ICM_INST(T)                                                          \
    template void launch_forces<T>(const Batch<T>&, hipStream_t);            \
    template void launch_dp2_sum<T>(const Batch<T>&, hipStream_t);           \
    template void launch_jps_table<T>(const Batch<T>&, hipStream_t);
ICM_INST(float)
ICM_INST(double)
#undef ICM_INST

}  // namespace icm
