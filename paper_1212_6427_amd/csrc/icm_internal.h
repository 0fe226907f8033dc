// Internal interfaces between the ICM context (api.hip) and the kernel
// launchers (fft.hip, grid.hip, blobs.hip). Everything here works on raw
// device pointers and one HIP stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "icm_common.h"

namespace icm {

constexpr int kMaxStages = 16;

// Workgroups of the right-hand-side kernel: a tile of kRhsTileX x kRhsTileY
// (x, y) columns and a z-chunk of GridDesc::zc planes (see RhsBlobs)
constexpr int kRhsTileX = 32, kRhsTileY = 16;
constexpr int kRhsZChunk = 16;    // default z-chunk (planes)
constexpr int kRhsZChunkMin = 4;  // smallest z-chunk: sizes the bins
__host__ __device__ inline int max_chunks(int nz) { return (nz + kRhsZChunkMin - 1) / kRhsZChunkMin; }
__host__ __device__ inline int rhs_tiles_x(int nx) { return (nx + kRhsTileX - 1) / kRhsTileX; }
__host__ __device__ inline int rhs_tiles_y(int ny) { return (ny + kRhsTileY - 1) / kRhsTileY; }
// bin slots: one per (tile, chunk) of the finest chunking, then the overflow
// count
__host__ __device__ inline int rhs_bins(int nx, int ny, int nz) {
    return rhs_tiles_x(nx) * rhs_tiles_y(ny) * max_chunks(nz);
}

// Mixed-radix (2, 3, 4, 8) Stockham plan of one FFT length.
struct FFTPlan {
    int n;
    int nst;
    int radix[kMaxStages];
};

// Field buffers of one replica. Real face fields hold 3 components of
// ncell values (x fastest); the spectrum holds 3 components of
// nz * ny rows of W = nx/2 + 1 complex values (kx fastest) at row pitch Wp,
// except on the fast FFT path, whose rows hold the nx/2 modes kx < nx/2 and
// whose Nyquist column kx = nx/2 is the separate array nyq (c, z, y).
template <typename T>
struct GridDesc {
    int nx, ny, nz, W;
    int Wp;            // spectrum row pitch (a multiple of 128 bytes; >= W, or
                       // >= nx/2 on the fast path)
    int fast;          // 1: register-resident FFT passes (all three N supported)
    int By, Bz;        // kx columns per block of the fast y and z passes
    int xt;            // threads per block of the fast x passes
    int zsmall;        // 1: the z pass holds the smaller per-thread plan (FP32)
    int zc;            // z planes per chunk of the right-hand-side kernel and its
                       // blob bins (4, 8 or 16; chosen per batch)
    long long ncell;   // nx * ny * nz
    long long nspec;   // nz * ny * Wp (per component)
    double h;
    double hs;         // half shift s / (2h) of the split three-point kernel
                       // (four-node layout); 0: the plain kernel
    T* v;              // fluid velocity v^n / v^{n+1}
    T* rhs;            // right-hand side / spread scratch field
    T* aux;            // inertial-correction field (dv~, dv)
    cplx<T>* spec;     // spectral work buffer
    cplx<T>* nyq;      // fast path: Nyquist column, 3 x nz x ny; else null
    // FFT plans and twiddles exp(-2 pi i m / N), m < N, per axis
    FFTPlan px, py, pz;
    const cplx<T>* twx;
    const cplx<T>* twy;
    const cplx<T>* twz;
    // difference symbols: Dhat_a = (e^{i theta} - 1)/h, lam_a = |Dhat_a|^2
    const cplx<T>* dx_hat;  // W entries
    const cplx<T>* dy_hat;  // ny entries
    const cplx<T>* dz_hat;  // nz entries
    const T* lx;
    const T* ly;
    const T* lz;
    // advection (NULL when off): the advective term of the previous step,
    // and a flag that is 1 once it holds one
    T* adv;
    unsigned int* adv_hist;
    // FP32-grid replicas: the k = 0 mode (mean velocity) carried in FP64.
    // k0[0..2] mean of v, k0[3..5] sum of the blob forces F of the step,
    // k0[6..8] sum of dp - m_e g (step 6); NULL in FP64 replicas
    double* k0;
    // Few-blob replicas on grids up to 128^3: the real-space kernel of the
    // discrete projection, K[(b * 3 + a) * ncell + cell] = (P e_b)_a at cell,
    // e_b the unit impulse on face 0 of component b (shared by the replicas
    // of one grid shape; P does not depend on h); NULL otherwise
    const T* ptab;
};

// Mixed-radix plan of one FFT length (radix 8, then 4, 2, 3); false if N
// has another prime factor or needs more than kMaxStages stages.
inline bool factor_plan(int n, FFTPlan& pl) {
    pl.n = n;
    pl.nst = 0;
    int m = n;
    while (m % 8 == 0 && pl.nst < kMaxStages) { pl.radix[pl.nst++] = 8; m /= 8; }
    while (m % 4 == 0 && pl.nst < kMaxStages) { pl.radix[pl.nst++] = 4; m /= 4; }
    while (m % 2 == 0 && pl.nst < kMaxStages) { pl.radix[pl.nst++] = 2; m /= 2; }
    while (m % 3 == 0 && pl.nst < kMaxStages) { pl.radix[pl.nst++] = 3; m /= 3; }
    return m == 1;
}

template <typename T>
bool fast_fft_available(int nx, int ny, int nz);

// Shape fields of a grid descriptor (sizes, spectrum pitch, FFT plans and
// the default launch shapes); the buffer and table pointers are left alone.
template <typename T>
void grid_shape(GridDesc<T>& g, const int32_t n[3], double h) {
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    g.W = g.nx / 2 + 1;
    g.fast = fast_fft_available<T>(g.nx, g.ny, g.nz) ? 1 : 0;
    // Launch shapes of the fast FFT passes (icm_autotune may change them):
    // 128 bytes of kx columns per y / z block, 256 threads per x block, the
    // smaller per-thread z plan.
    g.By = 128 / (int)sizeof(cplx<T>);
    g.Bz = 128 / (int)sizeof(cplx<T>);
    g.xt = 256;
    g.zsmall = 1;
    g.zc = kRhsZChunk;
    g.ncell = (long long)g.nx * g.ny * g.nz;
    // rows of the fast path hold kx < nx/2 (the Nyquist column has an array
    // of its own), so that at nx = 256 they carry no padding
    const int align = 128 / (int)sizeof(cplx<T>);
    const int cols = g.fast ? g.nx / 2 : g.W;
    g.Wp = (cols + align - 1) / align * align;
    g.nspec = (long long)g.nz * g.ny * g.Wp;
    g.h = h;
    factor_plan(g.nx, g.px);
    factor_plan(g.ny, g.py);
    factor_plan(g.nz, g.pz);
}

// Spectral multiplier applied between the forward and inverse transforms:
// w = P-hat( R-hat * scale / (a + b lambda) ), lambda = -L-hat >= 0.
struct SolveCoef {
    double a, b, scale;
};

// Physical constants of the right-hand side of step 2 (Sec. III.C).
struct RhsCoef {
    double rho_dt;      // rho / dt
    double half_eta_h2; // (eta / 2) / h^2
    double noise;       // (kT eta / (h^3 dt))^(1/2) / h, 0 = deterministic
    double adv;         // rho / h: scale of the advective flux differences
    double body[3];
    NoiseKey key;
};

// Blobs spread inside the right-hand-side kernel. stc holds, per blob and
// component a, the wrapped base nodes (as doubles) of the P-tap stencil on
// the a-component grid, the P weights of each axis, and the P derivative
// weights phi'(d)/h along axis a (kStcPerComp values per component).
// Blobs are binned by workgroup of the RHS kernel, i.e. by (tile, z-chunk):
// bin t = (chunk * tiles_y + tile_y) * tiles_x + tile_x lists bin_count[t]
// blobs at bin_list[t * kRhsTileCap]. A bin's blobs beyond kRhsTileCap go to
// the overflow list as (blob, bin) pairs, which launch_spread_overflow
// spreads with atomics.

constexpr int kRhsTileCap = 128;
constexpr int kStcPerComp = 3 + 4 * 4;
struct RhsBlobs {
    int nb;
    int kernel;
    const double* stc;       // nb * 3 * kStcPerComp
    const double* F;         // nb * 3 forces (spread with S)
    const double* cdrift;    // nb drift coefficients kT m~_f / m~ (NULL = no drift)
    int* bin_count;          // rhs_bins
    int* bin_list;           // rhs_bins * kRhsTileCap
    int* ovf_count;          // 1
    int* ovf_list;           // 2 * ovf_cap ints (blob, bin)
    int ovf_cap;
};

// ----------------------------------------------------------- blob buffers
struct BlobParams {
    int nb;
    double dt, rho, eta, kT;
    double box[3];
    double wca_eps, wca_sigma;
    double spring_k, spring_c[3];
    int slip;
};

struct BlobBufs {
    double *q, *u, *me, *fconst, *lag;     // state
    double *qh, *qw, *F, *Jn, *Jhvn, *Jhvt, *du, *dp, *dp2, *g, *Jhvnew;  // per step
    double* JLvt;                          // J L v~ (step 4 from the spectrum)
    double *c5, *cdrift;                   // per-blob coefficients
    unsigned int* flag;                    // numeric error flag
    // spread inside the right-hand-side kernel
    double* stc;                           // max_nb * 3 * kStcPerComp
    int* bin_count;                        // rhs_bins + 1 (the last is the overflow count)
    int* bin_list;                         // rhs_bins * kRhsTileCap
    int* ovf_list;                         // 2 * ovf_cap
    int ovf_cap;
};

// Cell list of the pair forces: n[a] cells of width >= the cutoff per axis
// (at least 3), heads[cell] = (stamp << kHeadBlobBits | first blob),
// next[blob]. The stamp is the step number + 1 modulo 2^40, so heads left by
// earlier steps read as empty. With heads == NULL the forces use the
// all-pairs kernel.
constexpr int kHeadBlobBits = 24;
__host__ __device__ __forceinline__ unsigned long long cell_stamp(unsigned long long step) {
    return (step + 1) & ((1ULL << (64 - kHeadBlobBits)) - 1);
}
struct CellGrid {
    int n[3];
    double inv_size[3];
    unsigned long long* heads;
    int* next;
};

// Selectors of per-replica arrays, resolved on the device.
enum FieldSel { kFieldV = 0, kFieldRhs = 1, kFieldAux = 2 };
enum BlobSel { kBlobNone = -1, kBlobQ = 0, kBlobQh, kBlobDp, kBlobDp2, kBlobC5, kBlobJhvt, kBlobG, kBlobLag };
enum SolveSel { kSolveH1 = 0, kSolveP = 1, kSolveH2 = 2 };

template <typename T>
__host__ __device__ __forceinline__ T* field_of(const GridDesc<T>& g, int sel) {
    return sel == kFieldV ? g.v : (sel == kFieldRhs ? g.rhs : g.aux);
}

__host__ __device__ __forceinline__ double* blob_of(const BlobBufs& b, int sel) {
    switch (sel) {
        case kBlobQ: return b.q;
        case kBlobQh: return b.qh;
        case kBlobDp: return b.dp;
        case kBlobDp2: return b.dp2;
        case kBlobC5: return b.c5;
        case kBlobJhvt: return b.Jhvt;
        case kBlobG: return b.g;
        case kBlobLag: return b.lag;
        default: return nullptr;
    }
}

// Everything a kernel needs to know about one replica. The descriptors of a
// context live in one device array; the replicas of a batch (same grid shape,
// kernel and inertial path) are contiguous there, and a batched launch finds
// its replica from the grid. The only value that changes from step to step is
// the device step counter, so a captured step replays unchanged.
template <typename T>
struct RepDesc {
    GridDesc<T> g;
    RhsCoef rc;                 // rc.key.step_* unused: see *step
    RhsBlobs rb;
    BlobParams bp;
    BlobBufs bb;
    CellGrid cg;
    SolveCoef solve[3];         // indexed by SolveSel
    int pair_mode;              // 0 no pair forces, 1 cell list, 2 all pairs
    unsigned long long* step;   // step counter n (incremented at the end of the step)
};

// Sum over nb blobs of a 3-vector per blob, a[3i + c], or (DIFF) a[3i + c] -
// m[i] b[3i + c], by the first 256 threads of a workgroup (every thread of
// it calls this) in a fixed order (so the same inputs give the same sum);
// thread 0 writes out[0..2]. Thread t adds blobs t, t + 256, t + 512, ...
// in that order, U per pass with all of a pass's loads issued before the
// first is added (at clamped indices, so that no branch stands between
// them).
template <bool DIFF, int U = DIFF ? 4 : 16>  // 7 or 3 loads per blob
__device__ inline void block_sum3(int nb, const double* a, const double* m, const double* b, double* out) {
    constexpr int NT = 256;
    __shared__ double red[3][NT];
    const int tid = (int)threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    if (tid < NT) {
        for (int i0 = 0; i0 < nb; i0 += U * NT) {
            double v[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * NT + tid;
                const int ic = i < nb ? i : nb - 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) v[u][c] = DIFF ? a[3 * ic + c] - m[ic] * b[3 * ic + c] : a[3 * ic + c];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + u * NT + tid < nb)
#pragma unroll
                    for (int c = 0; c < 3; ++c) s[c] += v[u][c];
            }
        }
        for (int c = 0; c < 3; ++c) red[c][tid] = s[c];
    }
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (tid < off)
            for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + off];
        __syncthreads();
    }
    if (tid == 0)
        for (int c = 0; c < 3; ++c) out[c] = red[c][0];
}

// The distinct tiles (runs of `span` nodes, the last run possibly shorter)
// of an axis of n nodes that the P-node stencil runs from wrapped base nodes
// b0 and b1 meet. The two runs overlap or touch (b1 is b0 or b0 - 1 modulo
// n), so together they cover at most P + 1 <= 5 consecutive nodes, which
// cross at most two tile starts: at most three tiles, and three only when a
// short last tile lies between them. Unused slots are -1.
template <int P>
__device__ __forceinline__ void axis_tiles(int b0, int b1, int n, int span, int& c0, int& c1, int& c2) {
    c0 = b0 / span;
    c1 = -1;
    c2 = -1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int t = 0; t < P; ++t) {
            int node = (r == 0 ? b0 : b1) + t;
            if (node >= n) node -= n;
            const int c = node / span;
            if (c != c0 && c != c1 && c != c2) {
                if (c1 < 0)
                    c1 = c;
                else
                    c2 = c;
            }
        }
    }
}

// Lists blob b of replica R (no-op for b >= nb) in every RHS bin (tile and
// z-chunk) its stencils meet, from the stencil records of the step-1 gather
// (per axis, the base node of the component grid offset by 0 along it and
// that of the two offset by h/2); a bin's entries beyond kRhsTileCap go to
// the overflow list. The counts start at zero: the previous step's final
// gather (or the host) cleared them. A record the step has not written yet
// (the autotuner's timing before a first step) may hold anything: a value
// outside the axis reads as node 0, so that every bin index stays in range.
template <typename T, int P>
__device__ inline void bin_blob_from_records(const RepDesc<T>& R, int b) {
    const RhsBlobs& rb = R.rb;
    if (b >= rb.nb) return;
    const int nx = R.g.nx, ny = R.g.ny, nz = R.g.nz, zc = R.g.zc;
    const int tiles_x = rhs_tiles_x(nx), tiles_y = rhs_tiles_y(ny);
    // record of component a: o + a kStcPerComp, base node along axis ax at [ax]
    const gptr<const double> o = as_global(rb.stc) + (long long)b * 3 * kStcPerComp;
    auto node = [](double d, int n) { return (d >= 0.0 && d < (double)n) ? (int)d : 0; };
    int x0, x1, x2, y0, y1, y2, z0, z1, z2;
    axis_tiles<P>(node(o[0], nx), node(o[kStcPerComp], nx), nx, kRhsTileX, x0, x1, x2);
    axis_tiles<P>(node(o[kStcPerComp + 1], ny), node(o[2 * kStcPerComp + 1], ny), ny, kRhsTileY, y0, y1, y2);
    axis_tiles<P>(node(o[2 * kStcPerComp + 2], nz), node(o[2], nz), nz, zc, z0, z1, z2);
    const gptr<int> count = as_global(rb.bin_count), list = as_global(rb.bin_list);
#pragma unroll
    for (int iz = 0; iz < 3; ++iz) {
        const int cz = iz == 0 ? z0 : (iz == 1 ? z1 : z2);
        if (cz < 0) continue;
#pragma unroll
        for (int iy = 0; iy < 3; ++iy) {
            const int cy = iy == 0 ? y0 : (iy == 1 ? y1 : y2);
            if (cy < 0) continue;
#pragma unroll
            for (int ix = 0; ix < 3; ++ix) {
                const int cx = ix == 0 ? x0 : (ix == 1 ? x1 : x2);
                if (cx < 0) continue;
                const int bin = (cz * tiles_y + cy) * tiles_x + cx;
                const int slot = __hip_atomic_fetch_add(&count[bin], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (slot < kRhsTileCap) {
                    list[(long long)bin * kRhsTileCap + slot] = b;
                } else {
                    const int os = __hip_atomic_fetch_add(as_global(rb.ovf_count), 1, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                    if (os < rb.ovf_cap) {
                        as_global(rb.ovf_list)[2 * os] = b;
                        as_global(rb.ovf_list)[2 * os + 1] = bin;
                    }
                }
            }
        }
    }
}

// The k = 0 mode of a step's solve when the replica carries its mean
// velocity in FP64 (called by the one thread that holds mode 0, after the
// solve, before the inverse transforms; the inverse transforms are
// unnormalised, so mode 0 becomes the mean of the output field).
//   H1 (step 2): the mean of v~ is the mean of v^n plus (dt/rho)(sum F / V +
//                f_body): spread forces keep their sum, while the viscous,
//                stochastic, drift and advective terms have none.
//   H2 (step 6): the mean of dv is sum (dp - m_e J dv~) / (rho V).
// In both cases the carried mean advances by the same amount, so the total
// momentum rho V mean + sum m_e u changes by exactly dt (sum F + V f_body).
template <typename T>
__device__ __forceinline__ void carry_mean_mode(const RepDesc<T>& R, int solve, cplx<T>& w0, cplx<T>& w1,
                                                cplx<T>& w2) {
    double* k0 = R.g.k0;
    const double vol = (double)R.g.ncell * R.g.h * R.g.h * R.g.h;
    double m[3];
    if (solve == kSolveH1) {
        for (int c = 0; c < 3; ++c) {
            m[c] = k0[c] + (k0[3 + c] / vol + R.rc.body[c]) / R.rc.rho_dt;
            k0[c] = m[c];
        }
    } else {
        for (int c = 0; c < 3; ++c) {
            m[c] = k0[6 + c] / (R.bp.rho * vol);
            k0[c] += m[c];
        }
    }
    w0 = cplx<T>{(T)m[0], (T)0};
    w1 = cplx<T>{(T)m[1], (T)0};
    w2 = cplx<T>{(T)m[2], (T)0};
}

// Host view of a batch: the device descriptors and the shape they share.
template <typename T>
struct Batch {
    const RepDesc<T>* d;  // nrep device descriptors
    int nrep;
    GridDesc<T> g;        // grid of the first replica (shape, FFT choice)
    int kernel;           // 3 or 4
    int max_nb;           // largest blob count of the batch
    bool any_cells, any_all_pairs;
    const RepDesc<T>* one;  // host copy of the descriptor when nrep == 1 (else NULL)
};

// ------------------------------------------------------------------- FFT
// Forward transform of field `in` (all three components), the spectral
// solve P-hat / (a + b lambda) with the replica's coefficients `solve`, and
// the inverse transform into field `out` (added to it with accumulate).
template <typename T>
void launch_fft_x_forward(const Batch<T>& B, int in, hipStream_t s);
template <typename T>
void launch_fft_y(const Batch<T>& B, int dir, hipStream_t s);
// carry: the solve of a step (H1 or H2) in a replica whose mean velocity is
// carried in FP64 (GridDesc::k0): the k = 0 mode is set from the carried
// mean and the exactly known change of total momentum, and the carry advanced.
template <typename T>
void launch_fft_z_solve(const Batch<T>& B, int solve, bool project, hipStream_t s, bool carry = false);
// accumulate: 0 writes field `out`, 1 adds to it, kXinvAlsoV (with out =
// kFieldAux) writes it and also adds the result to v.
constexpr int kXinvAlsoV = 2;
template <typename T>
void launch_fft_x_inverse(const Batch<T>& B, int out, int accumulate, hipStream_t s);

// Register-resident passes for N in {16, 32, 48, 64, 128, 256, 512};
// return false (launching nothing) for other sizes.
template <typename T>
bool fast_fft_available(int nx, int ny, int nz);
template <typename T>
bool fast_fft_y(const Batch<T>& B, int dir, hipStream_t s);
template <typename T>
bool fast_fft_z_solve(const Batch<T>& B, int solve, bool project, hipStream_t s, bool carry = false);
// The z pass and solve with its input spectrum formed from the blobs instead
// of read: the transform of S dp2 (step 6), so that no field is zeroed and
// spread and no x or y forward pass runs; with accumulate, the result is
// added to the spectrum already there. False (launching nothing) without a
// register-resident plan for the grid.
template <typename T>
bool fast_fft_z_solve_from_blobs(const Batch<T>& B, int solve, hipStream_t s, bool carry, bool accumulate);
template <typename T>
bool fast_fft_x_forward(const Batch<T>& B, int in, hipStream_t s);
template <typename T>
bool fast_fft_x_inverse(const Batch<T>& B, int out, int accumulate, hipStream_t s);

// ------------------------------------------------------------ grid kernels
template <typename T>
void launch_rhs(const Batch<T>& B, hipStream_t s);
template <typename T>
void launch_spread_overflow(const Batch<T>& B, hipStream_t s);
// rhs field of every replica = equilibrium sample N(0, sd^2) per face
// (noise key of step 0).
template <typename T>
void launch_equilibrium_noise(const Batch<T>& B, double sd, hipStream_t s);
template <typename T>
void launch_zero(const Batch<T>& B, int field, hipStream_t s);
// rhs -= 3/2 A^n - 1/2 A^{n-1} with A = D.(rho v v^T) of v; A^n kept in adv
// (replicas of a batch with advection on).
template <typename T>
void launch_advect(const Batch<T>& B, hipStream_t s);

// spread: field += h^-3 * prod(phi) * val at positions q, val_a = F[b][a] *
// (coef ? coef[b] : 1).
template <typename T>
void launch_spread(const Batch<T>& B, int field, int q, int F, int coef, hipStream_t s);
// gather: out[b][a] = sum prod(phi) f_a (or of (L f)_a with laplacian = true)
// at positions q; epi = kEpiDp / kEpiDp2 adds the per-component work of the
// inertial correction that uses the gathered value (step 4: du and dp;
// step 5: dp2 and, for m_e != 0, u^{n+1}).
enum GatherEpi { kEpiNone = 0, kEpiDp = 1, kEpiDp2 = 2 };
template <typename T>
void launch_gather(const Batch<T>& B, int field, int q, int out, bool laplacian, hipStream_t s,
                   int epi = kEpiNone);

// Fused gathers of the step (one 16-lane group per blob component): J^n v^n
// with the predictor and J^{n+1/2} v^n with the stencil records of
// q^{n+1/2} (step 1); J^{n+1/2} v^{n+1} with the position update (step 9,
// which also clears the RHS bin counters, advances the step counter and,
// in the first n_me replicas, gathers the lagged term J L dv from aux).
template <typename T>
void launch_gather_step1(const Batch<T>& B, hipStream_t s);
template <typename T>
void launch_gather_final(const Batch<T>& B, int n_me, bool lag_from_v, hipStream_t s);
// Bins of the RHS spread, one per RHS workgroup, from the stencil records
// (the step bins with the cell-list pair forces when the batch has them);
// counters must start at zero.
template <typename T>
void launch_bins(const Batch<T>& B, hipStream_t s);
// Stencil records at the positions q^n, as step 1 writes them at q^{n+1/2}:
// for the autotuner's RHS timing, whose bins need records before a first
// step has written any (the next step overwrites them).
template <typename T>
void launch_stencil_records(const Batch<T>& B, hipStream_t s);

// ------------------------------------------------------------ reductions
// acc[0..2] += rho h^3 sum v; acc[3] += rho h^3 sum v^2 / 2;
// acc[4] = max |v| (as bits), acc[5] = max |Dv| (as bits)
template <typename T>
void launch_field_diag(const GridDesc<T>& g, double rho, double* acc, hipStream_t s);
// g.k0[0..2] = mean of g.v, reduced in FP64 (acc: 16 zeroed doubles of
// scratch); nothing for replicas without the carry.
template <typename T>
void launch_carry_init(const GridDesc<T>& g, double rho, double* acc, hipStream_t s);

// ----------------------------------------------------------- blob kernels
template <typename T>
void launch_forces(const Batch<T>& B, hipStream_t s);
// Step 4 from the spectrum the first solve's z pass left (its y and x
// inverse passes deferred): J v~ and J L v~ of every blob component, with
// du and dp as the step-4 gather forms them (register-resident grids).
template <typename T>
void launch_spectral_gather(const Batch<T>& B, hipStream_t s);
// With the FP64-carried mean velocity: the sum of dp - m_e g per replica
// (after g came from the field path of step 5).
template <typename T>
void launch_dp2_sum(const Batch<T>& B, hipStream_t s);
// Step 5 through the projection-kernel table: g = J P S (c5 dp) for every
// blob, without forming the field (batches whose replicas have ptab); then
// dp2, u^{n+1} of the blobs with m_e != 0 and the carried sum of dp2.
template <typename T>
void launch_jps_table(const Batch<T>& B, hipStream_t s);
constexpr int kTabMaxBlobs = 8;
constexpr long long kTabMaxCells = 128LL * 128 * 128;
void launch_blob_diag(int nb, const double* me, const double* u, double* acc, hipStream_t s);

}  // namespace icm
