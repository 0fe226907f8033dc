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
__device__ __forceinline__ NormalPair<T> bm(const LogTab& lt, uint32_t wa, uint32_t wb) {
    NormalPair<T> r;
    box_muller(wa, wb, r.a, r.b, lt);
    return r;
}

__global__ void k_clear_ints(int* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Value spread to one tap (ia, ib, ic) of component a of blob b:
// (F_a prod w + c_drift prod w') / h^3, w' = phi'/h along axis a.
template <typename T>
__device__ __forceinline__ double tap_value(const RhsBlobs& rb, gptr<const double> o, int b, int a, int ia, int ib,
                                            int ic, double inv_h3) {
    const double wx = o[3 + ia], wy = o[7 + ib], wz = o[11 + ic];
    double v = as_global(rb.F)[3 * b + a] * wx * wy * wz;
    if (rb.cdrift) {
        const double dx = a == 0 ? o[15 + ia] : wx;
        const double dy = a == 1 ? o[15 + ib] : wy;
        const double dz = a == 2 ? o[15 + ic] : wz;
        v += as_global(rb.cdrift)[b] * dx * dy * dz;
    }
    return v * inv_h3;
}

// Spread of the (blob, tile) pairs a tile could not hold, restricted to the
// tile's cells, with atomics. One 16-lane group per (pair, component);
// replica blockIdx.y.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_spread_overflow(const RepDesc<T>* __restrict__ rd, int tiles_x,
                                                             int tiles_y, int rtx, int rty) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    const RhsBlobs rb = rd[blockIdx.y].rb;
    if (rb.nb <= 0) return;
    const int npairs = min(*rb.ovf_count, rb.ovf_cap);
    const int P = rb.kernel;
    const double inv_h = 1.0 / g.h;
    const double inv_h3 = inv_h * inv_h * inv_h;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < npairs * 48; t += gridDim.x * blockDim.x) {
        const int grp = t >> 4, r = t & 15;
        const int pr = grp / 3, a = grp - 3 * (grp / 3);
        if (r >= P * P) continue;
        const int b = rb.ovf_list[2 * pr], tile = rb.ovf_list[2 * pr + 1];
        const int txi = tile % tiles_x, tyi = (tile / tiles_x) % tiles_y, tzi = tile / (tiles_x * tiles_y);
        const int i0 = txi * rtx, j0 = tyi * rty, k0 = tzi * g.zc;
        gptr<const double> o = as_global(rb.stc) + ((long long)b * 3 + a) * kStcPerComp;
        const int ib = r / P;
        const int y = ((int)o[1] + ib) % g.ny;
        if (y < j0 || y >= j0 + rty) continue;
        for (int ic = 0; ic < P; ++ic) {
            const int z = ((int)o[2] + ic) % g.nz;
            if (z < k0 || z >= k0 + g.zc) continue;
            const int ia = r % P;
            const int x = ((int)o[0] + ia) % g.nx;
            if (x < i0 || x >= i0 + rtx) continue;
            const double v = tap_value<T>(rb, o, b, a, ia, ib, ic, inv_h3);
            atomicAdd(&g.rhs[a * g.ncell + ((long long)z * g.ny + y) * g.nx + x], (T)v);
        }
    }
}

// Right-hand side of the unperturbed solve (Eq. (provisional_step-1)):
//   rhs_a = (rho/dt) v_a + (eta/2) (L v)_a + s (D_w Sigma-hat)_a + f_body,a
// with Sigma-hat = W + W^T realised as 2 W_aa at cell centres and
// sqrt(2) W_ab on edges.
//
// The kernel marches along z. A block owns a TX x TY tile of
// (x, y) columns and a chunk of ZC planes; each thread owns one column. Every
// cell's two Philox blocks are generated once: block 1 of plane k+1 is drawn
// one plane ahead (the x-z and y-z edge stresses of plane k+1 enter plane k),
// W_zz of plane k-1 is carried in a register, and the in-plane neighbours'
// stresses and velocities are shared through LDS. Only the tile's one-cell
// halo ring regenerates the few normals it needs.
constexpr int RTX = kRhsTileX, RTY = kRhsTileY;

// ONE: a batch of one replica whose descriptor comes by value in the kernel
// arguments (constant memory the compiler may re-read at will); otherwise the
// replica's descriptor is read from the device array.
// sum_slice: one more z-slice of workgroups (the first), which sum the blob
// forces of the batch's replicas (fixed order) for the FP64-carried mean
// velocity of an FP32 grid (the z pass reads them); the pair forces are
// complete before this launch.
template <typename T, bool ONE>
__global__ void __launch_bounds__(RTX * RTY) k_rhs_march(const RepDesc<T>* __restrict__ rd, const RepDesc<T> one,
                                                        int ntz, int sum_slice) {
    __shared__ int s_blobs[kRhsTileCap];   // blobs of this workgroup's bin
    // Plane buffers, two of each: plane k uses buffer k - k0 mod 2, so the
    // next plane's writes never meet this plane's reads and one barrier per
    // plane suffices (plane k + 2 writes only after every thread has passed
    // the barrier of plane k + 1, hence finished reading plane k).
    __shared__ T s_acc2[2][3][RTY][RTX];       // spread accumulated for a plane
    __shared__ T sv2[2][3][RTY + 2][RTX + 2];  // velocity of a plane with halo
    __shared__ T sxx2[2][RTY][RTX + 1];        // W_xx, column 0 = i0 - 1
    __shared__ T sxy2[2][RTY + 1][RTX + 1];    // W_xy, row RTY = j0 + TY, column RTX = i0 + TX
    __shared__ T sxz2[2][RTY][RTX + 1];        // W_xz, column RTX = i0 + TX
    __shared__ T syy2[2][RTY + 1][RTX];        // W_yy, row 0 = j0 - 1
    __shared__ T syz2[2][RTY + 1][RTX];        // W_yz, row RTY = j0 + TY
    // the FP64 transform's logarithm table (the FP32 one uses the hardware
    // logarithm)
    LogTab lt{nullptr, nullptr};
    if constexpr (sizeof(T) == 8) {
        __shared__ double s_linv[kLogTab], s_lnf[kLogTab];
        fill_log_tab(s_linv, s_lnf);
        __syncthreads();
        lt = LogTab{s_linv, s_lnf};
    }
    const int tx = threadIdx.x % RTX, ty = threadIdx.x / RTX;
    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs,
    // so give XCD j a contiguous run of tiles (x fastest, then y, then z,
    // then replica): neighbouring tiles then share their halo lines in that
    // XCD's L2.
    const int ntx = gridDim.x, nty = gridDim.y;
    const int nzr = (int)gridDim.z - sum_slice;  // z-slices of tiles: chunks x replicas
    if (sum_slice && blockIdx.z == 0) {
        // the first slice, dispatched first, so that the sums overlap the tiles
        const int nrep = nzr / ntz;
        for (int r = blockIdx.x + ntx * blockIdx.y; r < nrep; r += ntx * nty) {
            const RepDesc<T>& Rr = ONE ? one : rd[r];
            block_sum3<false, 4>(Rr.bp.nb, Rr.bb.F, nullptr, nullptr, Rr.g.k0 + 3);  // few registers
        }
        return;
    }
    const int ntiles = ntx * nty * nzr;
    int tile = blockIdx.x + ntx * (blockIdx.y + nty * ((int)blockIdx.z - sum_slice));
    if (ntiles % 8 == 0) tile = (tile % 8) * (ntiles / 8) + tile / 8;
    const int tile_x = tile % ntx, tile_y = (tile / ntx) % nty, tile_zr = tile / (ntx * nty);
    const int rep = ONE ? 0 : tile_zr / ntz, tile_z = tile_zr - rep * ntz;
    const RepDesc<T>& R = ONE ? one : rd[rep];
    const GridDesc<T>& g = R.g;
    const RhsCoef& c = R.rc;
    const RhsBlobs& rb = R.rb;
    const unsigned long long step_n = *as_global(R.step);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const gptr<const T> gv = as_global((const T*)g.v);
    const gptr<T> grhs = as_global(g.rhs);
    const gptr<const double> gstc = as_global(rb.stc);
    const gptr<const double> gF = as_global(rb.F);
    const int i0 = tile_x * RTX, j0 = tile_y * RTY;
    const int k0 = tile_z * g.zc;
    const int k1 = min(k0 + g.zc, nz);
    const int i = i0 + tx, j = j0 + ty;
    const bool own = (i < nx) && (j < ny);
    const long long plane = (long long)nx * ny;
    const long long col = (long long)j * nx + i;
    const bool noisy = c.noise != 0.0;
    // The step words are uniform: keep them in scalar registers, so that the
    // uniform parts of the first Philox rounds run on the scalar unit.
    NoiseKey nk = c.key;
    nk.step_lo = __builtin_amdgcn_readfirstlane((uint32_t)step_n);
    nk.step_hi = __builtin_amdgcn_readfirstlane((uint32_t)(step_n >> 32));
    const T r2 = (T)1.41421356237309504880;
    // halo duty (valid tile extent; the right / top halo sits just past it,
    // wrapped): wave 0 takes the ring cells that need one Philox block per
    // plane (left column, bottom row), wave 1 those that need up to two
    // (right column, top row), so each of the two waves runs one halo branch
    // and their SIMDs carry similar extra work.
    static_assert(RTX + RTY <= 64, "one wave per half of the halo ring");
    const int wx = min(RTX, nx - i0), wy = min(RTY, ny - j0);
    const int tid = threadIdx.x;
    int hi = -1, hj = -1, hkind = -1;
    if (tid < RTY) { hkind = 0; hi = i0 - 1; hj = j0 + tid; }
    else if (tid < RTY + RTX) { hkind = 2; hi = i0 + tid - RTY; hj = j0 - 1; }
    else if (tid >= 64 && tid < 64 + RTY) { hkind = 1; hi = i0 + wx; hj = j0 + tid - 64; }
    else if (tid >= 64 + RTY && tid < 64 + RTY + RTX) { hkind = 3; hi = i0 + tid - 64 - RTY; hj = j0 + wy; }
    const int hiw = wrap(hi, nx), hjw = wrap(hj, ny);
    const bool hvalid = hkind >= 0 && (hkind >= 2 ? hi - i0 < wx : hj - j0 < wy);

    // registers carried along z. Cells (i, j, 2m) and (i, j, 2m+1) share the
    // Philox counter of pair m = i + Nx (j + Ny m); blocks A = 0, B = 1, C = 2:
    //   lower: A(0,1) -> xx, yy; A(2,3) -> zz, xy; B(0,1) -> xz, yz
    //   upper: B(2,3) -> xx, yy; C(0,1) -> zz, xy; C(2,3) -> xz, yz
    // An even plane draws A and C of its pair, an odd plane B of the next
    // pair (whose xz, yz enter the odd plane and whose xx, yy wait for the
    // pair's upper plane): three calls per two cells.
    // vr[s] and hr[s] are a ring of prefetch registers: see the march below
    T vr[4][3] = {}, hr[2][3] = {};
    T wzz_m = 0, wxz_c = 0, wyz_c = 0;
    T up_xx = 0, up_yy = 0, up_zz = 0, up_xy = 0;  // upper-cell normals of the current pair
    const uint32_t pairs_plane = (uint32_t)plane;  // pair counters per pair of planes
    // v is read one plane ahead of its use (vp for plane k + 1 was loaded
    // during plane k - 1; the halo ring's values likewise), so the loads'
    // latency overlaps a whole plane of work. Every thread issues these
    // loads, with no branch around them: a thread outside a ragged tile
    // reads a clamped column, one without a halo duty the wrapped corner
    // (nx - 1, ny - 1) (one line for the wave). The compiler's wait counts
    // then follow the issue order, and a plane's use of its prefetched
    // values waits for none of the loads issued for later planes.
    const long long colc = (long long)min(j, ny - 1) * nx + min(i, nx - 1);
    const long long hcol = (long long)hjw * nx + hiw;
#pragma unroll
    for (int a = 0; a < 3; ++a) hr[0][a] = gv[a * g.ncell + (long long)k0 * plane + hcol];
    const int km = wrap(k0 - 1, nz);
    {
        const int k0p = k0 + 1 == nz ? 0 : k0 + 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vr[0][a] = gv[a * g.ncell + km * plane + colc];
            vr[1][a] = gv[a * g.ncell + (long long)k0 * plane + colc];
            vr[2][a] = gv[a * g.ncell + (long long)k0p * plane + colc];
        }
    }
    if (own) {
        if (noisy) {
            // W_zz of the odd plane k0 - 1 (C of the previous pair); xz, yz of
            // plane k0 and xx, yy of plane k0 + 1 (B of the first pair)
            const uint32_t mprev = (uint32_t)(km / 2), m0 = (uint32_t)(k0 / 2);
            const u32x4 wc = noise_words(nk, mprev * pairs_plane + (uint32_t)col, 2);
            wzz_m = bm<T>(lt, wc.x, wc.y).a;
            const u32x4 wb = noise_words(nk, m0 * pairs_plane + (uint32_t)col, 1);
            const NormalPair<T> q = bm<T>(lt, wb.x, wb.y), r = bm<T>(lt, wb.z, wb.w);
            wxz_c = q.a;
            wyz_c = q.b;
            up_xx = r.a;
            up_yy = r.b;
        }
    }
    // the blobs of this workgroup's bin (its tile and z-chunk), which k_bins
    // listed; those beyond kRhsTileCap are in the overflow list
    for (int a = 0; a < 3; ++a) s_acc2[0][a][ty][tx] = s_acc2[1][a][ty][tx] = (T)0;
    const int P = rb.kernel;
    int nloc = 0;
    if (rb.nb > 0) {
        const int bin = (tile_z * nty + tile_y) * ntx + tile_x;
        nloc = min(as_global(rb.bin_count)[bin], kRhsTileCap);
        if (tid < nloc) s_blobs[tid] = as_global(rb.bin_list)[(long long)bin * kRhsTileCap + tid];
    }
    __syncthreads();
    const double inv_h3 = 1.0 / (g.h * g.h * g.h);
    // This thread's first spread item (local blob, component, x-y tap) is
    // plane independent apart from its z weight: keep it in registers.
    bool it_ok = false;
    int it_a = 0, it_x = 0, it_y = 0, it_z0 = 0;
    T tv0 = 0, tv1 = 0, tv2 = 0, tv3 = 0;
    if (tid < nloc * 48) {
        const int lb = tid / 48, rem = tid - 48 * lb;
        const int a = rem >> 4, r = rem & 15;
        if (r < P * P) {
            const int b = s_blobs[lb];
            gptr<const double> o = gstc + ((long long)b * 3 + a) * kStcPerComp;
            const int ia = r % P, ib = r / P;
            int x = (int)o[0] + ia, y = (int)o[1] + ib;
            if (x >= nx) x -= nx;
            if (y >= ny) y -= ny;
            if (x >= i0 && x < i0 + wx && y >= j0 && y < j0 + wy) {
                it_ok = true;
                it_a = a;
                it_x = x - i0;
                it_y = y - j0;
                it_z0 = (int)o[2];
                const double wxv = o[3 + ia], wyv = o[7 + ib];
                const double it_f = gF[3 * b + a] * wxv * wyv * inv_h3;
                double it_d = 0, dz0 = 0, dz1 = 0, dz2 = 0, dz3 = 0;
                if (rb.cdrift) {
                    const double cx = a == 0 ? o[15 + ia] : wxv, cy = a == 1 ? o[15 + ib] : wyv;
                    it_d = as_global(rb.cdrift)[b] * cx * cy * inv_h3;
                    if (a == 2) { dz0 = o[15]; dz1 = o[16]; dz2 = o[17]; dz3 = o[18]; }
                    else { dz0 = o[11]; dz1 = o[12]; dz2 = o[13]; dz3 = o[14]; }
                }
                tv0 = (T)(it_f * o[11] + it_d * dz0);
                tv1 = (T)(it_f * o[12] + it_d * dz1);
                tv2 = (T)(it_f * o[13] + it_d * dz2);
                tv3 = (T)(it_f * o[14] + it_d * dz3);
            }
        }
    }

    // The march is unrolled by four so that the prefetch ring rotates by
    // renaming, not by register moves: plane k reads vm, v0, vp from three
    // slots of vr and loads plane k + 2 into the fourth, the halo values
    // alternate between the two slots of hr. A move would have to wait for
    // the load just issued; renamed, each load has a whole plane of work to
    // land. The planes past the chunk's end (uniform over the block) stop.
    for (int kb = k0; kb < k1; kb += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = kb + u;
            if (k >= k1) break;
            T(&vm)[3] = vr[u];
            T(&v0)[3] = vr[(u + 1) & 3];
            T(&vp)[3] = vr[(u + 2) & 3];
            T(&vq)[3] = vr[(u + 3) & 3];
            T(&hcur)[3] = hr[u & 1];
            T(&hq)[3] = hr[(u + 1) & 1];
            auto& s_acc = s_acc2[u & 1];
            auto& sv = sv2[u & 1];
            auto& sxx = sxx2[u & 1];
            auto& sxy = sxy2[u & 1];
            auto& sxz = sxz2[u & 1];
            auto& syy = syy2[u & 1];
            auto& syz = syz2[u & 1];
            const int kp = k + 1 == nz ? 0 : k + 1;
            T wxx = 0, wyy = 0, wzz = 0, wxy = 0, wxz_n = 0, wyz_n = 0;
            if (it_ok) {
                int ic = k - it_z0;
                if (ic < 0) ic += nz;
                if (ic < P) atomicAdd(&s_acc[it_a][it_y][it_x], ic == 0 ? tv0 : (ic == 1 ? tv1 : (ic == 2 ? tv2 : tv3)));
            }
            // further items (tiles met by more than 10 blobs) read their data here
            for (int it = tid + blockDim.x; it < nloc * 3 * 16; it += blockDim.x) {
                const int lb = it / 48, rem = it - 48 * lb;
                const int a = rem >> 4, r = rem & 15;
                if (r >= P * P) continue;
                const int b = s_blobs[lb];
                gptr<const double> o = gstc + ((long long)b * 3 + a) * kStcPerComp;
                int ic = k - (int)o[2];
                if (ic < 0) ic += nz;
                if (ic >= P) continue;
                const int ia = r % P, ib = r / P;
                int x = (int)o[0] + ia, y = (int)o[1] + ib;
                if (x >= nx) x -= nx;
                if (y >= ny) y -= ny;
                if (x < i0 || x >= i0 + wx || y < j0 || y >= j0 + wy) continue;
                const double v = tap_value<T>(rb, o, b, a, ia, ib, ic, inv_h3);
                atomicAdd(&s_acc[a][y - j0][x - i0], (T)v);
            }
            {
                // the chunk's last plane loads (unused) values of planes
                // this block has just read, which the cache still holds
                const bool more = k + 1 < k1;
                const int kq = !more ? kp : (kp + 1 == nz ? 0 : kp + 1);
                const long long hn = (long long)(more ? kp : k) * plane + hcol;
#pragma unroll
                for (int a = 0; a < 3; ++a) vq[a] = gv[a * g.ncell + (long long)kq * plane + colc];
#pragma unroll
                for (int a = 0; a < 3; ++a) hq[a] = gv[a * g.ncell + hn];
            }
            if (own) {
                if (noisy) {
                    if ((k & 1) == 0) {
                        const uint32_t ctr = (uint32_t)(k / 2) * pairs_plane + (uint32_t)col;
                        const u32x4 wa = noise_words(nk, ctr, 0);
                        const NormalPair<T> p0 = bm<T>(lt, wa.x, wa.y), p1 = bm<T>(lt, wa.z, wa.w);
                        wxx = p0.a;
                        wyy = p0.b;
                        wzz = p1.a;
                        wxy = p1.b;
                        const u32x4 wc = noise_words(nk, ctr, 2);
                        const NormalPair<T> p2 = bm<T>(lt, wc.x, wc.y), p3 = bm<T>(lt, wc.z, wc.w);
                        up_zz = p2.a;
                        up_xy = p2.b;
                        wxz_n = p3.a;
                        wyz_n = p3.b;
                    } else {
                        wxx = up_xx;
                        wyy = up_yy;
                        wzz = up_zz;
                        wxy = up_xy;
                        const uint32_t ctr = (uint32_t)(kp / 2) * pairs_plane + (uint32_t)col;
                        const u32x4 wb = noise_words(nk, ctr, 1);
                        const NormalPair<T> p0 = bm<T>(lt, wb.x, wb.y), p1 = bm<T>(lt, wb.z, wb.w);
                        wxz_n = p0.a;
                        wyz_n = p0.b;
                        up_xx = p1.a;
                        up_yy = p1.b;
                    }
                }
                for (int a = 0; a < 3; ++a) sv[a][ty + 1][tx + 1] = v0[a];
                sxx[ty][tx + 1] = wxx;
                sxy[ty][tx] = wxy;
                sxz[ty][tx] = wxz_c;
                syy[ty + 1][tx] = wyy;
                syz[ty][tx] = wyz_c;
            }
            if (hvalid) {
                // LDS slot of the halo cell (column/row index within the tile + 1)
                const int sy = hkind <= 1 ? hj - j0 + 1 : (hkind == 2 ? 0 : wy + 1);
                const int sx = hkind == 0 ? 0 : (hkind == 1 ? wx + 1 : hi - i0 + 1);
                for (int a = 0; a < 3; ++a) sv[a][sy][sx] = hcur[a];
                if (noisy) {
                    // the halo cell's pair counter; which words hold its normals
                    // depends on the parity of k (see the pair layout above)
                    const uint32_t hctr = (uint32_t)(k / 2) * pairs_plane + (uint32_t)((long long)hjw * nx + hiw);
                    const bool odd = (k & 1) != 0;
                    if (hkind == 0 || hkind == 2) {
                        // xx (left) or yy (bottom): A(0,1) on even planes, B(2,3) on odd
                        const u32x4 w = noise_words(nk, hctr, odd ? 1 : 0);
                        const NormalPair<T> pr = odd ? bm<T>(lt, w.z, w.w) : bm<T>(lt, w.x, w.y);
                        if (hkind == 0)
                            sxx[hj - j0][0] = pr.a;
                        else
                            syy[0][hi - i0] = pr.b;
                    } else {
                        // right: xy and xz; top: xy and yz. Even planes: xy from
                        // A(2,3), xz / yz from B(0,1); odd planes: all from C.
                        T exy, ez;
                        if (odd) {
                            const u32x4 w = noise_words(nk, hctr, 2);
                            exy = bm<T>(lt, w.x, w.y).b;
                            const NormalPair<T> q = bm<T>(lt, w.z, w.w);
                            ez = hkind == 1 ? q.a : q.b;
                        } else {
                            const u32x4 w = noise_words(nk, hctr, 0);
                            exy = bm<T>(lt, w.z, w.w).b;
                            const u32x4 w1 = noise_words(nk, hctr, 1);
                            const NormalPair<T> q = bm<T>(lt, w1.x, w1.y);
                            ez = hkind == 1 ? q.a : q.b;
                        }
                        if (hkind == 1) {
                            sxy[hj - j0][wx] = exy;
                            sxz[hj - j0][wx] = ez;
                        } else {
                            sxy[wy][hi - i0] = exy;
                            syz[wy][hi - i0] = ez;
                        }
                    }
                }
            }
            __syncthreads();
            if (own) {
                T out[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T lap = sv[a][ty + 1][tx] + sv[a][ty + 1][tx + 2] + sv[a][ty][tx + 1] + sv[a][ty + 2][tx + 1] +
                                  vm[a] + vp[a] - (T)6 * v0[a];
                    out[a] = (T)c.rho_dt * v0[a] + (T)c.half_eta_h2 * lap + (T)c.body[a];
                }
                if (noisy) {
                    const T s = (T)c.noise;
                    const T dx = (T)2 * (wxx - sxx[ty][tx]) + r2 * (sxy[ty + 1][tx] - wxy) + r2 * (wxz_n - wxz_c);
                    const T dy = r2 * (sxy[ty][tx + 1] - wxy) + (T)2 * (wyy - syy[ty][tx]) + r2 * (wyz_n - wyz_c);
                    const T dz = r2 * (sxz[ty][tx + 1] - wxz_c) + r2 * (syz[ty + 1][tx] - wyz_c) + (T)2 * (wzz - wzz_m);
                    out[0] += s * dx;
                    out[1] += s * dy;
                    out[2] += s * dz;
                }
                const long long cell = (long long)k * plane + col;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    out[a] += s_acc[a][ty][tx];
                    s_acc[a][ty][tx] = (T)0;
                    grhs[a * g.ncell + cell] = out[a];
                }
            }
            wzz_m = wzz;
            wxz_c = wxz_n;
            wyz_c = wyz_n;
        }
    }
}

// Equilibrium sample: every face N(0, sd^2) from Philox block 3 of the cell
// (words (w0,w1) -> (x, y) faces, (w2,w3) -> (z face, unused)), with the
// noise key of step 0; replica blockIdx.y.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_eq_noise(const RepDesc<T>* __restrict__ rd, double sd) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    NoiseKey nk = rd[blockIdx.y].rc.key;
    nk.step_lo = 0;
    nk.step_hi = 0;
    __shared__ double s_linv[kLogTab], s_lnf[kLogTab];
    fill_log_tab(s_linv, s_lnf);
    __syncthreads();
    const LogTab lt{s_linv, s_lnf};
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= g.ncell) return;
    const u32x4 w = noise_words(nk, (uint32_t)cell, 3);
    double a, b, cz, unused;
    box_muller(w.x, w.y, a, b, lt);
    box_muller(w.z, w.w, cz, unused, lt);
    g.rhs[cell] = (T)(sd * a);
    g.rhs[g.ncell + cell] = (T)(sd * b);
    g.rhs[2 * g.ncell + cell] = (T)(sd * cz);
}

template <typename T>
__global__ void k_zero(const RepDesc<T>* __restrict__ rd, int sel) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    T* p = field_of(rd[blockIdx.y].g, sel);
    const long long n = 3 * g.ncell;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// Advective term of step 2 (Eq. (provisional_step-1) with the Adams-Bashforth
// lag of Eq. (Adams_Bashforth)): A = D.(rho v v^T) at the three faces of cell
// (i, j, k) in the centred conservative form of the staggered grid. Fluxes:
// rho (v_a averaged along a)^2 at cell centres, and rho (v_b averaged along
// a)(v_a averaged along b) on the edges shared by a- and b-faces; component
// a takes the difference of its fluxes across its control volume. Then
// rhs -= 3/2 A^n - 1/2 A^{n-1} (A^{n-1} := A^n while *adv_hist is 0) and
// adv = A^n, each element read and rewritten by the thread that owns it.
// Threads (64 x 4) over (x, y); blockIdx.z = k + nz * replica. The 27
// neighbour loads per cell hit the caches for all but the cell's own
// values.
template <typename T>
__global__ void __launch_bounds__(256) k_advect(const RepDesc<T>* __restrict__ rd, int nz) {
    const int rep = (int)blockIdx.z / nz;
    const int k = (int)blockIdx.z - rep * nz;
    const GridDesc<T> g = rd[rep].g;
    const int i = (int)blockIdx.x * 64 + (int)threadIdx.x;
    const int j = (int)blockIdx.y * 4 + (int)threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const T c = (T)rd[rep].rc.adv;
    const int nx = g.nx, ny = g.ny;
    const long long sz = (long long)nx * ny;
    const long long o = (long long)k * sz + (long long)j * nx + i;
    // periodic neighbour offsets
    const long long xm = i == 0 ? nx - 1 : -1, xp = i == nx - 1 ? -(nx - 1) : 1;
    const long long ym = j == 0 ? (long long)(ny - 1) * nx : -(long long)nx;
    const long long yp = j == ny - 1 ? -(long long)(ny - 1) * nx : (long long)nx;
    const long long zm = k == 0 ? (long long)(nz - 1) * sz : -sz;
    const long long zp = k == nz - 1 ? -(long long)(nz - 1) * sz : sz;
    const gptr<const T> vx = as_global((const T*)g.v);
    const gptr<const T> vy = vx + g.ncell;
    const gptr<const T> vz = vy + g.ncell;
    const T X0 = vx[o], Xxm = vx[o + xm], Xxp = vx[o + xp], Xym = vx[o + ym], Xyp = vx[o + yp];
    const T Xzm = vx[o + zm], Xzp = vx[o + zp], Xxpym = vx[o + xp + ym], Xxpzm = vx[o + xp + zm];
    const T Y0 = vy[o], Yxm = vy[o + xm], Yxp = vy[o + xp], Yym = vy[o + ym], Yyp = vy[o + yp];
    const T Yzm = vy[o + zm], Yzp = vy[o + zp], Yxmyp = vy[o + xm + yp], Yypzm = vy[o + yp + zm];
    const T Z0 = vz[o], Zxm = vz[o + xm], Zxp = vz[o + xp], Zym = vz[o + ym], Zyp = vz[o + yp];
    const T Zzm = vz[o + zm], Zzp = vz[o + zp], Zxmzp = vz[o + xm + zp], Zymzp = vz[o + ym + zp];
    const T q = (T)0.25;
    // edge fluxes at this cell's own edges (shared by two components each)
    const T Fxy = q * (Y0 + Yxm) * (X0 + Xym);
    const T Fxz = q * (Z0 + Zxm) * (X0 + Xzm);
    const T Fyz = q * (Z0 + Zym) * (Y0 + Yzm);
    // x: centres i +- 1/2, edges at j + 1 and k + 1
    const T cxp = X0 + Xxp, cxm = Xxm + X0;
    const T Sx = q * (cxp * cxp - cxm * cxm) + q * (Yyp + Yxmyp) * (Xyp + X0) - Fxy +
                 q * (Zzp + Zxmzp) * (Xzp + X0) - Fxz;
    // y: centres j +- 1/2, edges at i + 1 and k + 1
    const T cyp = Y0 + Yyp, cym = Yym + Y0;
    const T Sy = q * (cyp * cyp - cym * cym) + q * (Xxp + Xxpym) * (Yxp + Y0) - Fxy +
                 q * (Zzp + Zymzp) * (Yzp + Y0) - Fyz;
    // z: centres k +- 1/2, edges at i + 1 and j + 1
    const T czp = Z0 + Zzp, czm = Zzm + Z0;
    const T Sz = q * (czp * czp - czm * czm) + q * (Xxp + Xxpzm) * (Zxp + Z0) - Fxz +
                 q * (Yyp + Yypzm) * (Zyp + Z0) - Fyz;
    const bool hist = *g.adv_hist != 0u;
    const gptr<T> rhs = as_global(g.rhs);
    const gptr<T> adv = as_global(g.adv);
    const T A[3] = {c * Sx, c * Sy, c * Sz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long e = o + (long long)a * g.ncell;
        const T prev = hist ? adv[e] : A[a];
        rhs[e] -= (T)1.5 * A[a] - (T)0.5 * prev;
        adv[e] = A[a];
    }
}

// Component grid origin along axis beta for component a: 0 if beta == a
// (faces normal to a), else 1/2 (cell centres).
__device__ __forceinline__ double comp_offset(int beta, int a) { return beta == a ? 0.0 : 0.5; }

// S: field_a += h^-3 phi(dx) phi(dy) phi(dz) val_a. A group of 16 lanes
// serves one (blob, component); lane r < P^2 owns the x-row of z-tap r / P and
// y-tap r mod P and adds its P values atomically (kernels of neighbouring
// blobs may overlap). Replica blockIdx.y.
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_spread(const RepDesc<T>* __restrict__ rd, int fsel, int qsel, int Fsel,
                                                    int csel) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    const BlobBufs bb = rd[blockIdx.y].bb;
    const int nb = rd[blockIdx.y].bp.nb;
    T* field = field_of(rd[blockIdx.y].g, fsel);
    const double* __restrict__ q = blob_of(rd[blockIdx.y].bb, qsel);
    const double* __restrict__ F = blob_of(rd[blockIdx.y].bb, Fsel);
    const double* __restrict__ coef = blob_of(rd[blockIdx.y].bb, csel);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = t >> 4, r = t & 15;
    const int b = grp / 3, a = grp - 3 * (grp / 3);
    if (b >= nb || r >= P * P) return;
    const int cz = r / P, cy = r - P * (r / P);
    const double inv_h = 1.0 / g.h;
    const double val = F[3 * b + a] * (coef ? coef[b] : 1.0) * inv_h * inv_h * inv_h;
    AxisStencil<P> sx;
    axis_stencil<P>(q[3 * b + 0] * inv_h - comp_offset(0, a), g.nx, false, inv_h, g.hs, sx);
    int ny_, nz_;
    double wy, wz;
    axis_tap<P>(q[3 * b + 1] * inv_h - comp_offset(1, a), g.ny, cy, false, inv_h, g.hs, ny_, wy);
    axis_tap<P>(q[3 * b + 2] * inv_h - comp_offset(2, a), g.nz, cz, false, inv_h, g.hs, nz_, wz);
    T* f = field + a * g.ncell + ((long long)nz_ * g.ny + ny_) * g.nx;
    const double wzy = wz * wy * val;
#pragma unroll
    for (int aa = 0; aa < P; ++aa) atomicAdd(&f[sx.node[aa]], (T)(wzy * sx.w[aa]));
}

// One 16-lane group's J for component a at position (qx,qy,qz), returned to
// every lane of the group: lane 1 + 4 ax + tt (ax < 3, tt < 4) evaluates the
// kernel weight of tap tt along axis ax (zero past P taps) and shares it
// through shuffles, and lane r < P^2 sums the x-row of z-tap r / P and y-tap
// r mod P.
template <typename T, int P>
__device__ __forceinline__ double gather_group(const GridDesc<T>& g, const T* __restrict__ field, const double* q3,
                                               int a, int r, bool active) {
    const double inv_h = 1.0 / g.h;
    int rb_node = 0;
    double rw = 0.0;
    if (active && r >= 1 && r <= 12) {
        const int ax = (r - 1) >> 2, tt = (r - 1) & 3;
        const int nax = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
        const double x = fold_coord(q3[ax] * inv_h - comp_offset(ax, a), nax);
        const int base = (int)((P == 3) ? floor(x + 0.5) : floor(x)) - 1;
        rb_node = wrap_node(base, nax);
        if (tt < P) rw = kern_w<P>(x - (double)(base + tt), g.hs);
    }
    double wx[4], wy4[4], wz4[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        wx[tt] = __shfl(rw, 1 + tt, 16);
        wy4[tt] = __shfl(rw, 5 + tt, 16);
        wz4[tt] = __shfl(rw, 9 + tt, 16);
    }
    const int bx = __shfl(rb_node, 1, 16), by = __shfl(rb_node, 5, 16), bz = __shfl(rb_node, 9, 16);
    double acc = 0.0;
    if (active && r < P * P) {
        const int cz = r / P, cy = r - P * (r / P);
        int j = by + cy, k = bz + cz;
        if (j >= g.ny) j -= g.ny;
        if (k >= g.nz) k -= g.nz;
        const double wy = cy == 0 ? wy4[0] : (cy == 1 ? wy4[1] : (cy == 2 ? wy4[2] : wy4[3]));
        const double wz = cz == 0 ? wz4[0] : (cz == 1 ? wz4[1] : (cz == 2 ? wz4[2] : wz4[3]));
        const T* f = field + a * g.ncell + ((long long)k * g.ny + j) * g.nx;
        double s = 0.0;
#pragma unroll
        for (int aa = 0; aa < P; ++aa) {
            int x = bx + aa;
            if (x >= g.nx) x -= g.nx;
            s += wx[aa] * (double)f[x];
        }
        acc = wz * wy * s;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    return acc;
}

// gather_group at the positions whose stencil records k_gather_step1 wrote
// (o: the record of component a): the same wrapped nodes and weights, read
// instead of recomputed, so the result is the same to the bit.
template <typename T, int P>
__device__ __forceinline__ double gather_group_rec(const GridDesc<T>& g, const T* __restrict__ field,
                                                   gptr<const double> o, int a, int r, bool active) {
    double acc = 0.0;
    if (active && r < P * P) {
        const int cz = r / P, cy = r - P * (r / P);
        const int i0 = (int)o[0];
        int j = (int)o[1] + cy, k = (int)o[2] + cz;
        if (j >= g.ny) j -= g.ny;
        if (k >= g.nz) k -= g.nz;
        const double wy = o[7 + cy], wz = o[11 + cz];
        const T* f = field + a * g.ncell + ((long long)k * g.ny + j) * g.nx;
        double s = 0.0;
#pragma unroll
        for (int aa = 0; aa < P; ++aa) {
            int x = i0 + aa;
            if (x >= g.nx) x -= g.nx;
            s += o[3 + aa] * (double)f[x];
        }
        acc = wz * wy * s;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    return acc;
}

// The same with the field value at each node replaced by its 7-point
// Laplacian (periodic), for the lagged term J L dv.
template <typename T, int P>
__device__ __forceinline__ double gather_group_rec_lap(const GridDesc<T>& g, const T* __restrict__ field,
                                                       gptr<const double> o, int a, int r, bool active) {
    double acc = 0.0;
    if (active && r < P * P) {
        const int cz = r / P, cy = r - P * (r / P);
        const int nx = g.nx, ny = g.ny, nz = g.nz;
        const int i0 = (int)o[0];
        int j = (int)o[1] + cy, k = (int)o[2] + cz;
        if (j >= ny) j -= ny;
        if (k >= nz) k -= nz;
        const int jp = j + 1 == ny ? 0 : j + 1, jm = j == 0 ? ny - 1 : j - 1;
        const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
        const double inv_h = 1.0 / g.h;
        const double wy = o[7 + cy], wz = o[11 + cz];
        const T* f = field + a * g.ncell;
        const long long row = ((long long)k * ny + j) * nx;
        double s = 0.0;
#pragma unroll
        for (int aa = 0; aa < P; ++aa) {
            int i = i0 + aa;
            if (i >= nx) i -= nx;
            const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
            const double c0 = (double)f[row + i];
            const double l = ((double)f[row + ip] + (double)f[row + im] + (double)f[((long long)k * ny + jp) * nx + i] +
                              (double)f[((long long)k * ny + jm) * nx + i] + (double)f[((long long)kp * ny + j) * nx + i] +
                              (double)f[((long long)km * ny + j) * nx + i] - 6.0 * c0) *
                             inv_h * inv_h;
            s += o[3 + aa] * l;
        }
        acc = wz * wy * s;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    return acc;
}

// Step 1 fused, one 16-lane group per (blob, component) and five whole
// blobs per 256-thread workgroup (groups 0..14), so that a blob's three
// components meet at the workgroup barrier:
//  (a) Jn = J(q^n) v^n, q^{n+1/2} = q^n + dt/2 Jn, the one-body forces at
//      q^{n+1/2} and the position folded into the box (for the pair forces);
//  (b) Jhvn = J(q^{n+1/2}) v^n, with the stencil record of component a at
//      q^{n+1/2} (wrapped base nodes, the P weights of each axis, the
//      derivative weights along axis a) for the spread inside the RHS kernel
//      and the gathers of step 9, and the blob's insertion into its cell's
//      list for the pair forces.
constexpr int kStep1Blobs = kThreads / 48;
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_gather_step1(const RepDesc<T>* __restrict__ rd) {
    __shared__ double s_qh[3 * kStep1Blobs], s_qw[3 * kStep1Blobs];
    const GridDesc<T> g = rd[blockIdx.y].g;
    const BlobParams bp = rd[blockIdx.y].bp;
    const BlobBufs bb = rd[blockIdx.y].bb;
    const int grp = (int)threadIdx.x >> 4, r = (int)threadIdx.x & 15;
    const int lb = grp / 3, a = grp - 3 * (grp / 3);
    const int b = (int)blockIdx.x * kStep1Blobs + lb;
    const bool active = grp < 3 * kStep1Blobs && b < bp.nb;
    // (a)
    const double J = gather_group<T, P>(g, g.v, active ? bb.q + 3 * b : bb.q, a, r, active);
    if (active && r == 0) {
        const int i = 3 * b + a;
        bb.Jn[i] = J;
        const double qh = bb.q[i] + 0.5 * bp.dt * J;
        if (!isfinite(qh)) atomicOr(bb.flag, 1u);
        bb.qh[i] = qh;
        // (component a's box length and spring centre by select: a runtime
        // index into the parameter copy would put it in scratch memory)
        const double L = a == 0 ? bp.box[0] : (a == 1 ? bp.box[1] : bp.box[2]);
        const double cs = a == 0 ? bp.spring_c[0] : (a == 1 ? bp.spring_c[1] : bp.spring_c[2]);
        double f = bb.fconst[i];
        if (bp.spring_k != 0.0) f -= bp.spring_k * (qh - cs);
        bb.F[i] = f;
        const double qw = qh - L * floor(qh / L);
        bb.qw[i] = qw;
        s_qh[grp] = qh;
        s_qw[grp] = qw;
    }
    __syncthreads();
    // (b): lane 1 + 4 ax + tt computes (and stores) tap tt of axis ax of
    // the record; the group's gather reads the weights from those lanes
    const double inv_h = 1.0 / g.h;
    const int n[3] = {g.nx, g.ny, g.nz};
    int rb_node = 0;
    double rw = 0.0;
    if (active && r >= 1 && r <= 12) {
        const int ax = (r - 1) >> 2, tt = (r - 1) & 3;
        double* o = bb.stc + ((long long)b * 3 + a) * kStcPerComp;
        const double x = fold_coord(s_qh[3 * lb + ax] * inv_h - (ax == a ? 0.0 : 0.5), n[ax]);
        const int base = (int)((P == 3) ? floor(x + 0.5) : floor(x)) - 1;
        rb_node = wrap_node(base, n[ax]);
        if (tt == 0) o[ax] = (double)rb_node;
        const double d = x - (double)(base + tt);
        rw = (tt < P) ? kern_w<P>(d, g.hs) : 0.0;
        o[3 + 4 * ax + tt] = rw;
        if (ax == a) o[15 + tt] = (tt < P) ? kern_dw<P>(d, g.hs) * inv_h : 0.0;
    }
    double wx[4], wy4[4], wz4[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        wx[tt] = __shfl(rw, 1 + tt, 16);
        wy4[tt] = __shfl(rw, 5 + tt, 16);
        wz4[tt] = __shfl(rw, 9 + tt, 16);
    }
    const int bx = __shfl(rb_node, 1, 16), by = __shfl(rb_node, 5, 16), bz = __shfl(rb_node, 9, 16);
    // lane r < P^2 sums the x-row of z-tap r / P and y-tap r mod P, as
    // gather_group does, with the same nodes and weights
    double acc = 0.0;
    if (active && r < P * P) {
        const int cz = r / P, cy = r - P * (r / P);
        int j = by + cy, k = bz + cz;
        if (j >= g.ny) j -= g.ny;
        if (k >= g.nz) k -= g.nz;
        const double wy = cy == 0 ? wy4[0] : (cy == 1 ? wy4[1] : (cy == 2 ? wy4[2] : wy4[3]));
        const double wz = cz == 0 ? wz4[0] : (cz == 1 ? wz4[1] : (cz == 2 ? wz4[2] : wz4[3]));
        const T* f = g.v + a * g.ncell + ((long long)k * g.ny + j) * g.nx;
        double sx = 0.0;
#pragma unroll
        for (int aa = 0; aa < P; ++aa) {
            int x = bx + aa;
            if (x >= g.nx) x -= g.nx;
            sx += wx[aa] * (double)f[x];
        }
        acc = wz * wy * sx;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (!active) return;
    if (r == 0) bb.Jhvn[3 * b + a] = acc;
    // a head holds (stamp << kHeadBlobBits | blob) with the step's stamp, so
    // heads left by earlier steps read as empty and are never cleared
    if (r == 4 && a == 0 && rd[blockIdx.y].pair_mode == 1) {
        const CellGrid cg = rd[blockIdx.y].cg;
        int ci[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int cc = (int)(s_qw[3 * lb + ax] * cg.inv_size[ax]);
            ci[ax] = cc >= cg.n[ax] ? cg.n[ax] - 1 : (cc < 0 ? 0 : cc);
        }
        const unsigned long long stamp = cell_stamp(*rd[blockIdx.y].step);
        const long long cell = ((long long)ci[2] * cg.n[1] + ci[1]) * cg.n[0] + ci[0];
        const unsigned long long mine = (stamp << kHeadBlobBits) | (unsigned long long)b;
        const unsigned long long old = atomicExch(&cg.heads[cell], mine);
        cg.next[b] = ((old >> kHeadBlobBits) == stamp) ? (int)(old & ((1u << kHeadBlobBits) - 1)) : -1;
    }
}

// Stencil records at q^n: one thread per (blob, component), the same
// nodes, weights and derivative weights that k_gather_step1 records at
// q^{n+1/2}.
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_stencil_records(const RepDesc<T>* __restrict__ rd) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    const BlobParams bp = rd[blockIdx.y].bp;
    const BlobBufs bb = rd[blockIdx.y].bb;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / 3, a = t - 3 * (t / 3);
    if (b >= bp.nb) return;
    const double inv_h = 1.0 / g.h;
    const int n[3] = {g.nx, g.ny, g.nz};
    double* o = bb.stc + ((long long)b * 3 + a) * kStcPerComp;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const double x = fold_coord(bb.q[3 * b + ax] * inv_h - (ax == a ? 0.0 : 0.5), n[ax]);
        const int base = (int)((P == 3) ? floor(x + 0.5) : floor(x)) - 1;
        o[ax] = (double)wrap_node(base, n[ax]);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            const double d = x - (double)(base + tt);
            o[3 + 4 * ax + tt] = (tt < P) ? kern_w<P>(d, g.hs) : 0.0;
            if (ax == a) o[15 + tt] = (tt < P) ? kern_dw<P>(d, g.hs) * inv_h : 0.0;
        }
    }
}

// The RHS bins of a batch's replicas, one thread per blob (a batch with
// cell-list pair forces bins them in that launch instead; the autotuner's
// RHS timing uses this one).
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_bins(const RepDesc<T>* __restrict__ rd) {
    bin_blob_from_records<T, P>(rd[blockIdx.y], blockIdx.x * blockDim.x + threadIdx.x);
}

// Step 9 fused: Jhvnew = J(q^{n+1/2}) v^{n+1}; q^{n+1} = q^n + dt/2
// (Jhvnew + Jhvn); u^{n+1} = Jhvnew for m_e = 0 blobs; numeric flag on
// NaN/Inf or a displacement above h. In the first n_me replicas (those on
// the inertial path) also the lagged term J^{n+1/2} L dv of the next step's
// slip correction: from dv in aux, or (lag_from_v) as J L v^{n+1} - J L v~
// with J L v~ from step 4. The replica's blocks clear its RHS bins for the
// next step, and its first thread advances the step counter (no other kernel
// of the step reads the counter after the RHS).
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_gather_final(const RepDesc<T>* __restrict__ rd, int n_clear,
                                                          int n_me, int lag_from_v) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    const BlobParams bp = rd[blockIdx.y].bp;
    const BlobBufs bb = rd[blockIdx.y].bb;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = t; i < n_clear; i += gridDim.x * blockDim.x) bb.bin_count[i] = 0;
    if (t == 0) {
        *rd[blockIdx.y].step += 1;
        if (g.adv_hist) *g.adv_hist = 1u;  // this step's advective term is the next one's lag
    }
    const int grp = t >> 4, r = t & 15;
    const int b = grp / 3, a = grp - 3 * (grp / 3);
    const bool active = b < bp.nb;
    // J(q^{n+1/2}) v^{n+1} from the stencil records of this step's positions
    const gptr<const double> o = as_global((const double*)bb.stc) + ((long long)(active ? b : 0) * 3 + a) * kStcPerComp;
    const double J = gather_group_rec<T, P>(g, g.v, o, a, r, active);
    const bool inertial = (int)blockIdx.y < n_me;
    const double lag = inertial ? gather_group_rec_lap<T, P>(g, lag_from_v ? g.v : g.aux, o, a, r, active) : 0.0;
    if (active && r == 0) {
        const int i = 3 * b + a;
        if (inertial) bb.lag[i] = lag_from_v ? lag - bb.JLvt[i] : lag;
        bb.Jhvnew[i] = J;
        const double dq = 0.5 * bp.dt * (J + bb.Jhvn[i]);
        const double qn = bb.q[i] + dq;
        if (!isfinite(qn)) atomicOr(bb.flag, 1u);
        if (fabs(dq) > g.h) atomicOr(bb.flag, 2u);
        bb.q[i] = qn;
        if (bb.me[b] == 0.0) bb.u[i] = J;
    }
}

// J: out[b][a] = sum phi(dx) phi(dy) phi(dz) f_a (FP64 accumulation), one
// 16-lane group per (blob, component) reduced with shuffles; with lap = 1 the
// field value at each node is replaced by its 7-point Laplacian.
// With epi = kEpiDp (out = J^{n+1/2} v~, step 4): the slip correction du =
// [FULL] (J^{n+1/2} - J^n) v^n + [VISCOUS|FULL] (nu dt/2) c_lag and the
// excess momentum dp = m_e (u^n - J^{n+1/2} v~ - du); with epi = kEpiDp2
// (out = g = J dv~, step 5): the step-6 source dp2 = dp - m_e g and, for
// m_e != 0, u^{n+1} = J v~ + g + du (step 8).
template <typename T, int P>
__global__ void __launch_bounds__(kThreads) k_gather(const RepDesc<T>* __restrict__ rd, int fsel, int qsel, int osel,
                                                    int lap, int epi) {
    const GridDesc<T> g = rd[blockIdx.y].g;
    const BlobBufs bb = rd[blockIdx.y].bb;
    const int nb = rd[blockIdx.y].bp.nb;
    const T* __restrict__ field = field_of(rd[blockIdx.y].g, fsel);
    const double* __restrict__ q = blob_of(rd[blockIdx.y].bb, qsel);
    double* __restrict__ out = blob_of(rd[blockIdx.y].bb, osel);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int grp = t >> 4, r = t & 15;
    const int b = grp / 3, a = grp - 3 * (grp / 3);
    double acc = 0.0;
    if (b < nb && r < P * P) {
        const int cz = r / P, cy = r - P * (r / P);
        const double inv_h = 1.0 / g.h;
        AxisStencil<P> sx;
        axis_stencil<P>(q[3 * b + 0] * inv_h - comp_offset(0, a), g.nx, false, inv_h, g.hs, sx);
        int j, k;
        double wy, wz;
        axis_tap<P>(q[3 * b + 1] * inv_h - comp_offset(1, a), g.ny, cy, false, inv_h, g.hs, j, wy);
        axis_tap<P>(q[3 * b + 2] * inv_h - comp_offset(2, a), g.nz, cz, false, inv_h, g.hs, k, wz);
        const T* f = field + a * g.ncell;
        const int nx = g.nx, ny = g.ny, nz = g.nz;
        const long long row = ((long long)k * ny + j) * nx;
        double s = 0.0;
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
                val = ((double)f[row + ip] + (double)f[row + im] + (double)f[((long long)k * ny + jp) * nx + i] +
                       (double)f[((long long)k * ny + jm) * nx + i] + (double)f[((long long)kp * ny + j) * nx + i] +
                       (double)f[((long long)km * ny + j) * nx + i] - 6.0 * c0) *
                      inv_h * inv_h;
            }
            s += sx.w[aa] * val;
        }
        acc = wz * wy * s;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (b < nb && r == 0) {
        const int i = 3 * b + a;
        out[i] = acc;
        if (epi == kEpiDp) {
            const BlobParams bp = rd[blockIdx.y].bp;
            double du = 0.0;
            if (bp.slip == 2) du += bb.Jhvn[i] - bb.Jn[i];
            if (bp.slip >= 1) du += 0.5 * (bp.eta / bp.rho) * bp.dt * bb.lag[i];
            bb.du[i] = du;
            bb.dp[i] = bb.me[b] * (bb.u[i] - acc - du);
        } else if (epi == kEpiDp2) {
            const double me = bb.me[b];
            bb.dp2[i] = bb.dp[i] - me * acc;
            if (me != 0.0) bb.u[i] = bb.Jhvt[i] + acc + bb.du[i];
        }
    }
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
void launch_rhs(const Batch<T>& B, hipStream_t s) {
    const GridDesc<T>& g = B.g;
    const int ntz = (g.nz + g.zc - 1) / g.zc;
    const int sum_slice = (B.g.k0 && B.max_nb > 0) ? 1 : 0;
    const dim3 grid((unsigned)((g.nx + RTX - 1) / RTX), (unsigned)((g.ny + RTY - 1) / RTY),
                    (unsigned)(ntz * B.nrep + sum_slice));
    if (B.nrep == 1 && B.one)
        hipLaunchKernelGGL((k_rhs_march<T, true>), grid, dim3(RTX * RTY), 0, s, B.d, *B.one, ntz, sum_slice);
    else
        hipLaunchKernelGGL((k_rhs_march<T, false>), grid, dim3(RTX * RTY), 0, s, B.d, RepDesc<T>{}, ntz, sum_slice);
}

template <typename T>
void launch_spread_overflow(const Batch<T>& B, hipStream_t s) {
    // a tile's list holds kRhsTileCap blobs: with no more blobs in a replica
    // nothing can overflow, and the launch is skipped
    if (B.max_nb <= kRhsTileCap) return;
    const int tiles_x = (B.g.nx + RTX - 1) / RTX, tiles_y = (B.g.ny + RTY - 1) / RTY;
    hipLaunchKernelGGL(k_spread_overflow<T>, dim3(B.nrep > 8 ? 8 : 64, B.nrep), dim3(kThreads), 0, s, B.d, tiles_x,
                       tiles_y, RTX, RTY);
}

template <typename T>
void launch_equilibrium_noise(const Batch<T>& B, double sd, hipStream_t s) {
    hipLaunchKernelGGL(k_eq_noise<T>, dim3(grid_for(B.g.ncell), B.nrep), dim3(kThreads), 0, s, B.d, sd);
}

unsigned stream_blocks(long long n, int nrep) {
    long long b = (n + kThreads - 1) / kThreads;
    const long long cap = 4096 / (nrep > 0 ? nrep : 1) + 1;
    if (b > cap) b = cap;
    return (unsigned)(b < 1 ? 1 : b);
}

template <typename T>
void launch_zero(const Batch<T>& B, int field, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<T>, dim3(stream_blocks(3 * B.g.ncell, B.nrep), B.nrep), dim3(kThreads), 0, s, B.d,
                       field);
}

template <typename T>
void launch_advect(const Batch<T>& B, hipStream_t s) {
    // gridDim.z = planes x replicas stays within 65535: split large batches
    const int per = std::max(1, 65535 / B.g.nz);
    for (int r0 = 0; r0 < B.nrep; r0 += per) {
        const int nr = std::min(per, B.nrep - r0);
        const dim3 grid((unsigned)((B.g.nx + 63) / 64), (unsigned)((B.g.ny + 3) / 4), (unsigned)(B.g.nz * nr));
        hipLaunchKernelGGL(k_advect<T>, grid, dim3(64, 4), 0, s, B.d + r0, B.g.nz);
    }
}

template <typename T>
void launch_spread(const Batch<T>& B, int field, int q, int F, int coef, hipStream_t s) {
    if (B.max_nb <= 0) return;
    const dim3 grid(grid_for(48LL * B.max_nb), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_spread<T, 3>), grid, dim3(kThreads), 0, s, B.d, field, q, F, coef);
    else
        hipLaunchKernelGGL((k_spread<T, 4>), grid, dim3(kThreads), 0, s, B.d, field, q, F, coef);
}

template <typename T>
void launch_gather(const Batch<T>& B, int field, int q, int out, bool laplacian, hipStream_t s, int epi) {
    if (B.max_nb <= 0) return;
    const dim3 grid(grid_for(48LL * B.max_nb), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_gather<T, 3>), grid, dim3(kThreads), 0, s, B.d, field, q, out, laplacian ? 1 : 0, epi);
    else
        hipLaunchKernelGGL((k_gather<T, 4>), grid, dim3(kThreads), 0, s, B.d, field, q, out, laplacian ? 1 : 0, epi);
}

template <typename T>
void launch_gather_step1(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb <= 0) return;
    const dim3 grid((unsigned)((B.max_nb + kStep1Blobs - 1) / kStep1Blobs), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_gather_step1<T, 3>), grid, dim3(kThreads), 0, s, B.d);
    else
        hipLaunchKernelGGL((k_gather_step1<T, 4>), grid, dim3(kThreads), 0, s, B.d);
}

template <typename T>
void launch_stencil_records(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb <= 0) return;
    const dim3 grid((unsigned)((3 * B.max_nb + kThreads - 1) / kThreads), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_stencil_records<T, 3>), grid, dim3(kThreads), 0, s, B.d);
    else
        hipLaunchKernelGGL((k_stencil_records<T, 4>), grid, dim3(kThreads), 0, s, B.d);
}

template <typename T>
void launch_bins(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb <= 0) return;
    const dim3 grid((unsigned)((B.max_nb + kThreads - 1) / kThreads), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_bins<T, 3>), grid, dim3(kThreads), 0, s, B.d);
    else
        hipLaunchKernelGGL((k_bins<T, 4>), grid, dim3(kThreads), 0, s, B.d);
}

template <typename T>
void launch_gather_final(const Batch<T>& B, int n_me, bool lag_from_v, hipStream_t s) {
    // always launched: its first block per replica advances the step counter
    const int n_clear = rhs_bins(B.g.nx, B.g.ny, B.g.nz) + 1;  // every bin count and the overflow count
    const dim3 grid(grid_for(48LL * (B.max_nb > 0 ? B.max_nb : 1)), B.nrep);
    if (B.kernel == 3)
        hipLaunchKernelGGL((k_gather_final<T, 3>), grid, dim3(kThreads), 0, s, B.d, n_clear, n_me,
                           lag_from_v ? 1 : 0);
    else
        hipLaunchKernelGGL((k_gather_final<T, 4>), grid, dim3(kThreads), 0, s, B.d, n_clear, n_me,
                           lag_from_v ? 1 : 0);
}

__global__ void k_carry_from_sum(double* k0, const double* acc, double inv) {
    if (threadIdx.x < 3) k0[threadIdx.x] = acc[threadIdx.x] * inv;
}

template <typename T>
void launch_carry_init(const GridDesc<T>& g, double rho, double* acc, hipStream_t s) {
    if (!g.k0) return;
    launch_field_diag(g, rho, acc, s);
    hipLaunchKernelGGL(k_carry_from_sum, dim3(1), dim3(64), 0, s, g.k0, acc,
                       1.0 / (rho * g.h * g.h * g.h * (double)g.ncell));
}

template <typename T>
void launch_field_diag(const GridDesc<T>& g, double rho, double* acc, hipStream_t s) {
    long long b = (g.ncell + kThreads - 1) / kThreads;
    if (b > 2048) b = 2048;
    hipLaunchKernelGGL(k_field_diag<T>, dim3((unsigned)b), dim3(kThreads), 0, s, g, rho, acc);
}

#define ICM_INST(T)                                                                              \
    template void launch_rhs<T>(const Batch<T>&, hipStream_t);                                   \
    template void launch_spread_overflow<T>(const Batch<T>&, hipStream_t);                       \
    template void launch_equilibrium_noise<T>(const Batch<T>&, double, hipStream_t);             \
    template void launch_zero<T>(const Batch<T>&, int, hipStream_t);                             \
    template void launch_spread<T>(const Batch<T>&, int, int, int, int, hipStream_t);            \
    template void launch_gather<T>(const Batch<T>&, int, int, int, bool, hipStream_t, int);      \
    template void launch_field_diag<T>(const GridDesc<T>&, double, double*, hipStream_t);        \
    template void launch_carry_init<T>(const GridDesc<T>&, double, double*, hipStream_t);        \
    template void launch_gather_step1<T>(const Batch<T>&, hipStream_t);                          \
    template void launch_bins<T>(const Batch<T>&, hipStream_t);                                  \
    template void launch_stencil_records<T>(const Batch<T>&, hipStream_t);                       \
    template void launch_gather_final<T>(const Batch<T>&, int, bool, hipStream_t);               \
    template void launch_advect<T>(const Batch<T>&, hipStream_t);
ICM_INST(float)
ICM_INST(double)
#undef ICM_INST

}  // namespace icm
