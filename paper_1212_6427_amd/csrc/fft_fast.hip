// Register-resident FFT passes for the grid sizes of the paper's runs
// (N in {16, 32, 48, 64, 128, 256, 512}); other sizes use the LDS Stockham
// kernels of fft.hip.
//
// Layout of one line of length N on TL = N / E threads: thread t holds the E
// elements n = t + TL * i (i < E) in registers. A Stockham stage of radix R
// keeps this layout on input, so the first stage reads global memory in it
// and the last stage leaves the natural-order result in it; the stages in
// between exchange through LDS once each. With lines laid side by side along
// the contiguous kx axis (y and z passes) every global access is a run of B
// consecutive complex values (128 bytes), and the z pass keeps the three
// velocity components of a mode in one thread, so the Helmholtz divide and
// the 3x3 projection of Sec. III.D happen in registers between the forward
// and inverse transforms.
#include <algorithm>
#include <cstdlib>

#include "icm_internal.h"

namespace icm {

namespace {

constexpr size_t kLdsMax = 64 * 1024;

// ---------------------------------------------------------- register DFTs
template <typename T, int DIR>
__device__ __forceinline__ void rdft2(cplx<T>* v) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, int DIR>
__device__ __forceinline__ void rdft3(cplx<T>* v) {
    const T c = (T)0.86602540378443864676;
    const cplx<T> s = cadd(v[1], v[2]);
    const cplx<T> d = csub(v[1], v[2]);
    const cplx<T> t = {v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y};
    const cplx<T> id = cmul_i(d, DIR);
    v[0] = cadd(v[0], s);
    v[1] = {t.x + c * id.x, t.y + c * id.y};
    v[2] = {t.x - c * id.x, t.y - c * id.y};
}

template <typename T, int DIR>
__device__ __forceinline__ void rdft4(cplx<T>* v) {
    const cplx<T> t0 = cadd(v[0], v[2]);
    const cplx<T> t1 = csub(v[0], v[2]);
    const cplx<T> t2 = cadd(v[1], v[3]);
    const cplx<T> t3 = cmul_i(csub(v[1], v[3]), DIR);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

template <typename T, int DIR>
__device__ __forceinline__ void rdft8(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    rdft4<T, DIR>(e);
    rdft4<T, DIR>(o);
    const T r = (T)0.70710678118654752440;
    o[1] = {r * (o[1].x - DIR * o[1].y), r * (o[1].y + DIR * o[1].x)};
    o[2] = cmul_i(o[2], DIR);
    o[3] = {r * (-o[3].x - DIR * o[3].y), r * (-o[3].y + DIR * o[3].x)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v[m] = cadd(e[m], o[m]);
        v[m + 4] = csub(e[m], o[m]);
    }
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <typename T, int DIR>
__device__ __forceinline__ void rdft16(cplx<T>* v) {
    cplx<T> A[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cplx<T> w[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
        rdft4<T, DIR>(w);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) A[n2][k1] = w[k1];
    }
    // twiddles exp(DIR 2 pi i n2 k1 / 16)
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
    const T c2 = (T)0.70710678118654752440;
    const cplx<T> w1 = {c1, DIR * s1}, w2 = {c2, DIR * c2}, w3 = {s1, DIR * c1};
    const cplx<T> w6 = {-c2, DIR * c2}, w9 = {-c1, -DIR * s1};
    A[1][1] = cmul(A[1][1], w1);
    A[1][2] = cmul(A[1][2], w2);
    A[1][3] = cmul(A[1][3], w3);
    A[2][1] = cmul(A[2][1], w2);
    A[2][2] = cmul_i(A[2][2], DIR);
    A[2][3] = cmul(A[2][3], w6);
    A[3][1] = cmul(A[3][1], w3);
    A[3][2] = cmul(A[3][2], w6);
    A[3][3] = cmul(A[3][3], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> w[4] = {A[0][k1], A[1][k1], A[2][k1], A[3][k1]};
        rdft4<T, DIR>(w);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = w[k2];
    }
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void rdft(cplx<T>* v) {
    if constexpr (R == 2) rdft2<T, DIR>(v);
    if constexpr (R == 3) rdft3<T, DIR>(v);
    if constexpr (R == 4) rdft4<T, DIR>(v);
    if constexpr (R == 8) rdft8<T, DIR>(v);
    if constexpr (R == 16) rdft16<T, DIR>(v);
}

// One Stockham stage on the strided register layout. Butterfly j = t + TL m
// takes x[j + r N/R] (register m + M r), twiddles it by
// w^(r (j mod Ns)), w = exp(DIR 2 pi i / (Ns R)), and applies a radix-R DFT.
template <typename T, int N, int E, int R, int Ns, int DIR>
__device__ __forceinline__ void reg_stage(cplx<T> (&a)[E], int t, const cplx<T>* tw) {
    constexpr int TL = N / E, M = E / R;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        cplx<T> v[R];
        const int k = (t + TL * m) % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cplx<T> x = a[m + M * r];
            if constexpr (Ns > 1) {
                if (r > 0) {
                    cplx<T> w = tw[r * k * (N / (Ns * R))];
                    if (DIR > 0) w.y = -w.y;
                    x = cmul(x, w);
                }
            }
            v[r] = x;
        }
        rdft<T, R, DIR>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) a[m + M * r] = v[r];
    }
}

// Stage outputs go to y[(j / Ns) Ns R + j mod Ns + r Ns]; bring them back
// to the strided layout through LDS (element n at lds[n * ls + lo]).
// SK skews the LDS index (n -> n + n / 2^SK) so that lines stored
// contiguously (x pass, ls = 1) do not put a thread's consecutive outputs,
// which lanes write in lock step, into the same banks; SK >= 16 disables it.
template <int SK>
__device__ __forceinline__ int skew(int n) {
    if constexpr (SK >= 16) return n;
    else return n + (n >> SK);
}

// How the exchanges of one transform synchronise (reg_fft's SYNC):
//   kSyncBlock  workgroup barrier before the writes and after them;
//   kSyncFresh  as kSyncBlock without the barrier before the first exchange,
//               for a transform that is the first user of its LDS buffer;
//   kSyncWave   each line lies within one wave (TL divides 64 and lines are
//               consecutive lanes), whose LDS accesses complete in program
//               order: the compiler only must not move them across the wave
//               barrier.
constexpr int kSyncBlock = 0, kSyncFresh = 1, kSyncWave = 2;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int N, int E, int R, int Ns, int SK, int SYNC, bool FIRST>
__device__ __forceinline__ void reg_exchange(cplx<T> (&a)[E], int t, cplx<T>* lds, int ls, int lo) {
    constexpr int TL = N / E, M = E / R;
    if constexpr (SYNC == kSyncWave)
        wave_sync();
    else if constexpr (SYNC == kSyncBlock || !FIRST)
        __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = t + TL * m;
        const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[skew<SK>(base + r * Ns) * ls + lo] = a[m + M * r];
    }
    if constexpr (SYNC == kSyncWave)
        wave_sync();
    else
        __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = lds[skew<SK>(t + TL * i) * ls + lo];
}

template <typename T, int N, int E, int R0, int R1, int R2, int DIR, int SK = 16, int SYNC = kSyncBlock>
__device__ __forceinline__ void reg_fft(cplx<T> (&a)[E], int t, cplx<T>* lds, int ls, int lo, const cplx<T>* tw) {
    static_assert(SYNC != kSyncWave || (64 % (N / E) == 0), "a line within one wave");
    reg_stage<T, N, E, R0, 1, DIR>(a, t, tw);
    if constexpr (R1 > 1) {
        reg_exchange<T, N, E, R0, 1, SK, SYNC, true>(a, t, lds, ls, lo);
        reg_stage<T, N, E, R1, R0, DIR>(a, t, tw);
        if constexpr (R2 > 1) {
            reg_exchange<T, N, E, R1, R0, SK, SYNC, false>(a, t, lds, ls, lo);
            reg_stage<T, N, E, R2, R0 * R1, DIR>(a, t, tw);
        }
    }
}

// Line stride (in complex elements) of the x-pass LDS lines with skew.
template <int N>
constexpr int xline() { return N + N / 16 + 1; }

// The spectrum as a buffer resource (gfx9-family descriptor word 3); byte
// offsets are 32-bit, which covers 3 components of a 512^3 FP64 spectrum.
template <typename T>
struct SpecBuf {
    __amdgpu_buffer_rsrc_t r;
    __device__ SpecBuf(cplx<T>* base, unsigned long long bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)(uint32_t)bytes, 0x00020000)) {}
    __device__ cplx<T> load(uint32_t vo, uint32_t so) const {
        if constexpr (sizeof(T) == 4)
            return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
        else
            return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
    }
    __device__ void store(cplx<T> v, uint32_t vo, uint32_t so) const {
        if constexpr (sizeof(T) == 4) {
            typedef unsigned int u2 __attribute__((ext_vector_type(2)));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)vo, (int)so, 0);
        } else {
            typedef unsigned int u4 __attribute__((ext_vector_type(4)));
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, (int)vo, (int)so, 0);
        }
    }
};

// Two consecutive complex values (one dwordx4 access in FP32).
template <typename T>
struct alignas(2 * sizeof(cplx<T>)) CPair {
    cplx<T> v[2];
};

// 16 bytes of real values (one dwordx4 access).
template <typename T>
struct alignas(16) Vec16 {
    T v[16 / sizeof(T)];
};

template <typename T>
__device__ __forceinline__ void load_tw(cplx<T>* dst, const cplx<T>* src, int n) {
    const gptr<const cplx<T>> gs = as_global(src);
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = gs[i];
}

// Spectrum layout of the fast passes: rows of the nx/2 modes kx < nx/2 at
// pitch Wp (a multiple of 128 bytes), rows ordered (c, z, y); the Nyquist
// column kx = nx/2 in its own array nyq, ordered (c, z, y). At nx = 256 the
// rows then carry no padding, and the y and z passes work on full column
// tiles of B consecutive kx (each access of a wave a run of B complex
// values); tail blocks (grid column ceil((nx/2) / B)) transform the Nyquist
// column of B planes (y pass) or B ky rows (z pass) from the contiguous
// nyq array.

// ------------------------------------------------------------------ y pass
// Block: B consecutive kx < nx/2 of one (z, component) plane of replica
// blockIdx.z / 3, thread (b = tid mod B, t = tid / B); or, in the tail
// column of the grid, the Nyquist column of B planes, thread
// (b = tid / TL, t = tid mod TL) so that lanes read consecutive y.
template <typename T, int N, int E, int R0, int R1, int R2, int DIR>
__global__ void __launch_bounds__(512) k_y_fast(const RepDesc<T>* __restrict__ rd, int B) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tws = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* lds = tws + N;
    const GridDesc<T> g = rd[blockIdx.z / 3].g;
    constexpr int TL = N / E;
    const int H = g.nx / 2;
    const int comp = (int)(blockIdx.z % 3);
    int b, t;
    bool ok;
    gptr<cplx<T>> base;
    long long stride;
    if ((int)blockIdx.x < (H + B - 1) / B) {
        // B consecutive kx < nx/2 of plane z = blockIdx.y
        b = threadIdx.x % B;
        t = threadIdx.x / B;
        const int kx = blockIdx.x * B + b;
        ok = kx < H;
        base = as_global(g.spec) + (long long)comp * g.nspec + (long long)blockIdx.y * N * g.Wp + kx;
        stride = g.Wp;
    } else {
        // tail: the Nyquist column of planes blockIdx.y B + b, contiguous
        // along y in nyq, so consecutive lanes take consecutive y
        if ((int)blockIdx.y * B >= g.nz) return;
        b = threadIdx.x / TL;
        t = threadIdx.x % TL;
        const int z = blockIdx.y * B + b;
        ok = z < g.nz;
        base = as_global(g.nyq) + ((long long)comp * g.nz + z) * N;
        stride = 1;
    }
    load_tw(tws, g.twy, N);
    cplx<T> a[E];
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = ok ? base[(long long)(t + TL * i) * stride] : cplx<T>{0, 0};
    // the first stage takes no twiddles; the first exchange's barrier orders
    // the twiddle writes before the second stage reads them
    reg_fft<T, N, E, R0, R1, R2, DIR, 16, kSyncFresh>(a, t, lds, B, b, tws);
    if (ok) {
#pragma unroll
        for (int i = 0; i < E; ++i) base[(long long)(t + TL * i) * stride] = a[i];
    }
}

// --------------------------------------------------------- z pass + solve
// Block: B consecutive kx < nx/2 of one ky row of replica blockIdx.z, or, in
// the tail column of the grid, the Nyquist column of B ky rows; each thread
// (b = tid mod B, t = tid / B) holds all three components of its column, so
// the Helmholtz divide and the 3 x 3 projection of every mode happen in
// registers between the forward and inverse transforms.
// SRC: the input spectrum is not read but formed from the replica's blobs:
// the field S f (f = dp2, the source of step 6) is a sum of tensor-product
// stencils, so its discrete Fourier transform over (x, y, z) is, per blob and
// component c, h^-3 f_c times the product of three one-dimensional sums
// sum_m w_a[m] exp(-2 pi i k_a (base_a + m) / n_a) over the stencil's nodes
// (the same nodes and weights as the spread, from the stencil records).
// This replaces zeroing the field, spreading into it and the x and y
// forward passes for replicas with few blobs.
template <typename T, int N, int E>
__device__ __forceinline__ void spectral_source(const RepDesc<T>& R, int kx, int ky, int t, const cplx<T>* twz,
                                                cplx<T> (&a0)[E], cplx<T> (&a1)[E], cplx<T> (&a2)[E]) {
    constexpr int TL = N / E;
    const GridDesc<T>& g = R.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const gptr<const cplx<T>> twx = as_global(g.twx), twy = as_global(g.twy);
    const gptr<const double> stc = as_global((const double*)R.bb.stc);
    const gptr<const double> dp2 = as_global((const double*)R.bb.dp2);
    const double ih3 = 1.0 / (g.h * g.h * g.h);
#pragma unroll
    for (int i = 0; i < E; ++i) a0[i] = a1[i] = a2[i] = cplx<T>{0, 0};
    const int nb = R.bp.nb;
    for (int b = 0; b < nb; ++b) {
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            const double f = dp2[3 * b + c] * ih3;
            if (f == 0.0) continue;
            const gptr<const double> o = stc + ((long long)b * 3 + c) * kStcPerComp;
            // x and y factors: sum over the stencil's four nodes (weights past
            // the kernel's width are zero)
            cplx<T> wxs = {0, 0}, wys = {0, 0};
            int ix = (int)(((long long)kx * (long long)o[0]) % nx), iy = (int)(((long long)ky * (long long)o[1]) % ny);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const T wx = (T)o[3 + m], wy = (T)o[7 + m];
                const cplx<T> ex = twx[ix], ey = twy[iy];
                wxs = {wxs.x + wx * ex.x, wxs.y + wx * ex.y};
                wys = {wys.x + wy * ey.x, wys.y + wy * ey.y};
                ix += kx;
                if (ix >= nx) ix -= nx;
                iy += ky;
                if (iy >= ny) iy -= ny;
            }
            cplx<T> wxy = cmul(wxs, wys);
            wxy = {(T)f * wxy.x, (T)f * wxy.y};
            const T wz0 = (T)o[11], wz1 = (T)o[12], wz2 = (T)o[13], wz3 = (T)o[14];
            const int bz = (int)o[2];
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int kz = t + TL * i;
                int iz = (int)(((long long)kz * bz) % nz);
                cplx<T> wzs = {0, 0};
                const T wz[4] = {wz0, wz1, wz2, wz3};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const cplx<T> ez = twz[iz];
                    wzs = {wzs.x + wz[m] * ez.x, wzs.y + wz[m] * ez.y};
                    iz += kz;
                    if (iz >= nz) iz -= nz;
                }
                const cplx<T> v = cmul(wxy, wzs);
                if (c == 0) a0[i] = cadd(a0[i], v);
                if (c == 1) a1[i] = cadd(a1[i], v);
                if (c == 2) a2[i] = cadd(a2[i], v);
            }
        }
    }
}

// SRC 0: the input spectrum read; 1: formed from the blobs; 2: formed from the
// blobs and the result added to the spectrum already there.
// LDS: twiddles (N), the exchange buffer (N B), then the z symbols of the
// solve, d_z (N complex) and the Laplacian's eigenvalues (N), so that the
// solve reads them without a global-memory round trip per mode.
template <typename T, int N, int E, int R0, int R1, int R2, int SRC = 0>
__global__ void __launch_bounds__(512) k_z_fast(const RepDesc<T>* __restrict__ rd, int B, int solve,
                                                 int project) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tws = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* lds = tws + N;
    cplx<T>* sdz = lds + N * B;
    T* slz = reinterpret_cast<T*>(sdz + N);
    const GridDesc<T> g = rd[blockIdx.z].g;
    const SolveCoef sc = rd[blockIdx.z].solve[solve];
    const int b = threadIdx.x % B, t = threadIdx.x / B;
    const int H = g.nx / 2;
    const bool tail = (int)blockIdx.x >= (H + B - 1) / B;
    if (tail && (int)blockIdx.y * B >= g.ny) return;
    // main blocks: B consecutive kx < nx/2 of ky row blockIdx.y; tail
    // blocks: the Nyquist column of ky rows blockIdx.y B + b (nyq array)
    const int kx = tail ? H : (int)blockIdx.x * B + b;
    const int y = tail ? (int)blockIdx.y * B + b : (int)blockIdx.y;
    const bool ok = tail ? y < g.ny : kx < H;
    // The twiddle and solve tables. FP32: each thread's first entry is
    // loaded into registers before the column loads and written to LDS after
    // them, so that the table round trip overlaps the column loads (loads in
    // flight retire in order: the writes wait for the tables only); blocks
    // narrower than N load the rest afterwards. FP64 (whose pencils leave no
    // registers for that) stages them first.
    constexpr bool kLate = sizeof(T) == 4;
    const gptr<const cplx<T>> gtw = as_global(g.twz), gdz = as_global(g.dz_hat);
    const gptr<const T> glz = as_global(g.lz);
    if constexpr (!kLate) {
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            tws[i] = gtw[i];
            sdz[i] = gdz[i];
            slz[i] = glz[i];
        }
    }
    const int ti = min((int)threadIdx.x, N - 1);
    cplx<T> tw0{}, dz0{};
    T lz0 = 0;
    if constexpr (kLate) {
        tw0 = gtw[ti];
        dz0 = gdz[ti];
        lz0 = glz[ti];
    }
    auto stage_tables = [&]() {
        if constexpr (kLate) {
            if ((int)threadIdx.x < N) {
                tws[threadIdx.x] = tw0;
                sdz[threadIdx.x] = dz0;
                slz[threadIdx.x] = lz0;
            }
            for (int i = threadIdx.x + blockDim.x; i < N; i += blockDim.x) {
                tws[i] = gtw[i];
                sdz[i] = gdz[i];
                slz[i] = glz[i];
            }
        }
    };
    constexpr int TL = N / E;
    // Buffer accesses: one 32-bit per-thread offset (column, first plane); the
    // plane and component offsets are uniform and go in the scalar offset, so
    // the 3E loads and stores need no per-access address registers.
    constexpr uint32_t cs = (uint32_t)sizeof(cplx<T>);
    const unsigned long long ncol = (unsigned long long)g.nz * g.ny;  // Nyquist values per component
    const SpecBuf<T> sb(tail ? g.nyq : g.spec, 3ull * (tail ? ncol : (unsigned long long)g.nspec) * cs);
    const uint32_t zb = (uint32_t)(tail ? g.ny : g.ny * g.Wp) * cs;       // bytes between z planes
    const uint32_t cb = (uint32_t)(tail ? ncol : (unsigned long long)g.nspec) * cs;  // between components
    const uint32_t vo = tail ? ((uint32_t)t * (uint32_t)g.ny + (uint32_t)y) * cs
                             : ((uint32_t)t * (uint32_t)(g.ny * g.Wp) + (uint32_t)(y * g.Wp + kx)) * cs;
    // Loads are issued component by component, so that the transform of
    // component 0 can start while those of components 1 and 2 are still in
    // flight (the load counter retires in order). They are unconditional:
    // a column that does not exist reads row padding, another row or (past
    // the buffer's end) zero, transforms it on its own and is never stored,
    // so no select has to wait for the loads.
    cplx<T> a0[E], a1[E], a2[E];
    if constexpr (SRC > 0) {
        // the transform in (x, y, z) of the spread field, formed directly
        stage_tables();
        __syncthreads();  // twiddles in LDS
        spectral_source<T, N, E>(rd[blockIdx.z], kx, y, t, tws, a0, a1, a2);
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) a0[i] = sb.load(vo, (uint32_t)(TL * i) * zb);
#pragma unroll
        for (int i = 0; i < E; ++i) a1[i] = sb.load(vo, (uint32_t)(TL * i) * zb + cb);
#pragma unroll
        for (int i = 0; i < E; ++i) a2[i] = sb.load(vo, (uint32_t)(TL * i) * zb + 2 * cb);
        stage_tables();
        __syncthreads();
        reg_fft<T, N, E, R0, R1, R2, -1>(a0, t, lds, B, b, tws);
        reg_fft<T, N, E, R0, R1, R2, -1>(a1, t, lds, B, b, tws);
        reg_fft<T, N, E, R0, R1, R2, -1>(a2, t, lds, B, b, tws);
    }
    // the barrier after the loads (or after the spectral source's twiddles)
    // has ordered the table writes before these reads
    if (ok) {
        const T lxy = as_global(g.lx)[kx] + as_global(g.ly)[y];
        const cplx<T> dx = as_global(g.dx_hat)[kx], dy = as_global(g.dy_hat)[y];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int kz = t + TL * i;
            const T lam = lxy + slz[kz];
            T f;
            if constexpr (sizeof(T) == 4)  // hardware reciprocal (1 ulp) in FP32
                f = (T)sc.scale * __builtin_amdgcn_rcpf((T)sc.a + (T)sc.b * lam);
            else
                f = sc.scale / (sc.a + sc.b * lam);
            cplx<T> w0 = {a0[i].x * f, a0[i].y * f};
            cplx<T> w1 = {a1[i].x * f, a1[i].y * f};
            cplx<T> w2 = {a2[i].x * f, a2[i].y * f};
            if ((project & 1) && lam > (T)0) {
                const cplx<T> dz = sdz[kz];
                const cplx<T> d = cadd(cadd(cmul(dx, w0), cmul(dy, w1)), cmul(dz, w2));
                T il;
                if constexpr (sizeof(T) == 4)
                    il = __builtin_amdgcn_rcpf(lam);
                else
                    il = (T)1 / lam;
                const cplx<T> dd = {d.x * il, d.y * il};
                w0 = csub(w0, cmul(cconj(dx), dd));
                w1 = csub(w1, cmul(cconj(dy), dd));
                w2 = csub(w2, cmul(cconj(dz), dd));
            }
            a0[i] = w0;
            a1[i] = w1;
            a2[i] = w2;
        }
        // mode k = 0 (kx = ky = kz = 0: thread t = 0, register 0 of column 0)
        if ((project & 2) && g.k0 && !tail && kx == 0 && y == 0 && t == 0)
            carry_mean_mode(rd[blockIdx.z], solve, a0[0], a1[0], a2[0]);
    }
    // each component is stored as soon as its inverse transform is done
    auto put = [&](cplx<T>(&a)[E], uint32_t co) {
        if (!ok) return;
        if constexpr (SRC == 2) {
#pragma unroll
            for (int i = 0; i < E; ++i) a[i] = cadd(a[i], sb.load(vo, (uint32_t)(TL * i) * zb + co));
        }
#pragma unroll
        for (int i = 0; i < E; ++i) sb.store(a[i], vo, (uint32_t)(TL * i) * zb + co);
    };
    reg_fft<T, N, E, R0, R1, R2, 1>(a0, t, lds, B, b, tws);
    put(a0, 0);
    reg_fft<T, N, E, R0, R1, R2, 1>(a1, t, lds, B, b, tws);
    put(a1, cb);
    reg_fft<T, N, E, R0, R1, R2, 1>(a2, t, lds, B, b, tws);
    put(a2, 2 * cb);
}

// ------------------------------------------------------------------ x pass
// Block: P row pairs of component blockIdx.y mod 3 of replica blockIdx.y / 3;
// thread (t = tid mod TL, l = tid / TL).
// Rows 2p and 2p+1 are packed as z = a + i b; their half spectra are
// separated by Hermitian symmetry after the transform.
template <typename T, int N, int E, int R0, int R1, int R2>
__global__ void __launch_bounds__(512) k_xfwd_fast(const RepDesc<T>* __restrict__ rd, int in_sel, int P) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tws = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* lds = tws + N;
    const GridDesc<T> g = rd[blockIdx.y / 3].g;
    const gptr<const T> in = as_global((const T*)field_of(rd[blockIdx.y / 3].g, in_sel));
    const int c = (int)(blockIdx.y % 3);
    constexpr int TL = N / E;
    const int t = threadIdx.x % TL, l = threadIdx.x / TL;
    constexpr int H = N / 2;
    const long long npairs = (long long)g.ny * g.nz / 2;
    const long long p = (long long)blockIdx.x * P + l;
    const bool ok = p < npairs;
    load_tw(tws, g.twx, N);
    // stage the block's row pairs through LDS with contiguous loads
    const long long row0 = (long long)c * g.ncell + 2 * ((long long)blockIdx.x * P) * N;
    const long long lim = (long long)c * g.ncell + 2 * npairs * N;
    constexpr int LS = xline<N>();
    // 16-byte loads: V consecutive values of both rows per thread; each
    // thread takes NL such pieces (blockDim = P TL), all loads issued before
    // the first is consumed
    constexpr int V = 16 / (int)sizeof(T);
    static_assert((N / V) % TL == 0, "row pieces per thread");
    constexpr int NL = (N / V) / TL;
    Vec16<T> ra[NL], rb[NL];
#pragma unroll
    for (int m = 0; m < NL; ++m) {
        const int idx = threadIdx.x + m * blockDim.x;
        const int ll = idx / (N / V), x = (idx - ll * (N / V)) * V;
        const long long o = row0 + 2LL * ll * N + x;
        ra[m] = Vec16<T>{};
        rb[m] = Vec16<T>{};
        if (o < lim) {
            ra[m] = *(gptr<const Vec16<T>>)(in + o);
            rb[m] = *(gptr<const Vec16<T>>)(in + o + N);
        }
    }
#pragma unroll
    for (int m = 0; m < NL; ++m) {
        const int idx = threadIdx.x + m * blockDim.x;
        const int ll = idx / (N / V), x = (idx - ll * (N / V)) * V;
#pragma unroll
        for (int q = 0; q < V; ++q) lds[ll * LS + skew<4>(x + q)] = cplx<T>{ra[m].v[q], rb[m].v[q]};
    }
    __syncthreads();
    // from here on each line is touched only by its own TL lanes, which lie in
    // one wave: wave-level synchronisation suffices
    cplx<T> a[E];
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = lds[l * LS + skew<4>(t + TL * i)];
    reg_fft<T, N, E, R0, R1, R2, -1, 4, kSyncWave>(a, t, lds, 1, l * LS, tws);
    wave_sync();
#pragma unroll
    for (int i = 0; i < E; ++i) lds[l * LS + skew<4>(t + TL * i)] = a[i];
    wave_sync();
    if (!ok) return;
    const gptr<cplx<T>> d0 = as_global(g.spec) + (long long)c * g.nspec + 2 * p * g.Wp;
    // modes kx < N/2, two consecutive per thread (16-byte stores for FP32;
    // N/2 is even); the Nyquist mode kx = N/2 of both rows goes to nyq
    for (int k = 2 * t; k < H; k += 2 * TL) {
        CPair<T> ea, eb;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kk = k + q;
            const cplx<T> zk = lds[l * LS + skew<4>(kk)];
            const cplx<T> zc = cconj(lds[l * LS + skew<4>((N - kk) % N)]);
            const cplx<T> s = cadd(zk, zc), d = csub(zk, zc);
            ea.v[q] = {(T)0.5 * s.x, (T)0.5 * s.y};
            eb.v[q] = {(T)0.5 * d.y, (T)-0.5 * d.x};
        }
        *(gptr<CPair<T>>)(d0 + k) = ea;
        *(gptr<CPair<T>>)(d0 + g.Wp + k) = eb;
    }
    if (t == 0) {
        const cplx<T> zk = lds[l * LS + skew<4>(H)];
        const cplx<T> zc = cconj(zk);
        const cplx<T> s = cadd(zk, zc), d = csub(zk, zc);
        const gptr<cplx<T>> nq = as_global(g.nyq) + (long long)c * g.nz * g.ny + 2 * p;
        nq[0] = cplx<T>{(T)0.5 * s.x, (T)0.5 * s.y};
        nq[1] = cplx<T>{(T)0.5 * d.y, (T)-0.5 * d.x};
    }
}

template <typename T, int N, int E, int R0, int R1, int R2>
__global__ void __launch_bounds__(512) k_xinv_fast(const RepDesc<T>* __restrict__ rd, int out_sel, int P,
                                                    int accumulate) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* tws = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* lds = tws + N;
    const GridDesc<T> g = rd[blockIdx.y / 3].g;
    const gptr<T> out = as_global(field_of(rd[blockIdx.y / 3].g, out_sel));
    const int c = (int)(blockIdx.y % 3);
    constexpr int TL = N / E;
    constexpr int H = N / 2;
    const int t = threadIdx.x % TL, l = threadIdx.x / TL;
    const long long npairs = (long long)g.ny * g.nz / 2;
    const long long p = (long long)blockIdx.x * P + l;
    const bool ok = p < npairs;
    load_tw(tws, g.twx, N);
    const long long rp = g.Wp;
    // a line past the last row pair reads the first one (never stored), so
    // that no load sits behind a branch
    const long long pc = ok ? p : 0;
    const gptr<const cplx<T>> s0 = as_global((const cplx<T>*)g.spec) + (long long)c * g.nspec + 2 * pc * rp;
    constexpr int LS = xline<N>();
    // modes kx < N/2, two consecutive per thread (16-byte loads for FP32):
    // pairs k = 2t + 2 TL m, m < E/4, and the Nyquist mode of both rows
    // (from nyq, real parts only), all loads issued before the first is
    // consumed
    static_assert(E % 4 == 0 && 2 * TL * (E / 4) == H, "mode pairs per thread");
    constexpr int NP = E / 4;
    CPair<T> ea[NP], eb[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int k = 2 * t + 2 * TL * m;
        ea[m] = *(gptr<const CPair<T>>)(s0 + k);
        eb[m] = *(gptr<const CPair<T>>)(s0 + rp + k);
    }
    const gptr<const cplx<T>> nq = as_global((const cplx<T>*)g.nyq) + (long long)c * g.nz * g.ny + 2 * pc;
    const cplx<T> nyA = nq[0], nyB = nq[1];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int k = 2 * t + 2 * TL * m;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kk = k + q;
            cplx<T> A = ea[m].v[q], Bv = eb[m].v[q];
            if (kk == 0) {
                A.y = 0;
                Bv.y = 0;
            }
            lds[l * LS + skew<4>(kk)] = {A.x - Bv.y, A.y + Bv.x};
            if (kk > 0) lds[l * LS + skew<4>(N - kk)] = {A.x + Bv.y, -A.y + Bv.x};
        }
    }
    if (t == 0) lds[l * LS + skew<4>(H)] = {nyA.x, nyB.x};
    __syncthreads();  // twiddles
    // each line is transformed by its own TL lanes, which lie in one wave
    cplx<T> a[E];
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = lds[l * LS + skew<4>(t + TL * i)];
    reg_fft<T, N, E, R0, R1, R2, 1, 4, kSyncWave>(a, t, lds, 1, l * LS, tws);
    // unstage through LDS so that rows are written with contiguous stores
    wave_sync();
#pragma unroll
    for (int i = 0; i < E; ++i) lds[l * LS + skew<4>(t + TL * i)] = a[i];
    __syncthreads();
    const long long row0 = (long long)c * g.ncell + 2 * ((long long)blockIdx.x * P) * N;
    const long long lim = (long long)c * g.ncell + 2 * npairs * N;
    // 16-byte stores: V consecutive values of both rows per thread
    constexpr int V = 16 / (int)sizeof(T);
    for (int idx = threadIdx.x; idx < P * (N / V); idx += blockDim.x) {
        const int ll = idx / (N / V), x = (idx - ll * (N / V)) * V;
        const long long o = row0 + 2LL * ll * N + x;
        if (o >= lim) continue;
        Vec16<T> ra, rb;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const cplx<T> z = lds[ll * LS + skew<4>(x + q)];
            ra.v[q] = z.x;
            rb.v[q] = z.y;
        }
        const gptr<Vec16<T>> oa = (gptr<Vec16<T>>)(out + o);
        const gptr<Vec16<T>> ob = (gptr<Vec16<T>>)(out + o + N);
        if (accumulate == kXinvAlsoV) {
            // write the field and add it to v (v += dv of step 7)
            *oa = ra;
            *ob = rb;
            const gptr<Vec16<T>> va = (gptr<Vec16<T>>)(g.v + o);
            const gptr<Vec16<T>> vb = (gptr<Vec16<T>>)(g.v + o + N);
            Vec16<T> pa = *va, pb = *vb;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                pa.v[q] += ra.v[q];
                pb.v[q] += rb.v[q];
            }
            *va = pa;
            *vb = pb;
            continue;
        }
        if (accumulate) {
            const Vec16<T> pa = *oa, pb = *ob;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                ra.v[q] += pa.v[q];
                rb.v[q] += pb.v[q];
            }
        }
        *oa = ra;
        *ob = rb;
    }
}

// ------------------------------------------------ step 4 from the spectrum
// After the first solve's z pass the spectrum holds S(kx, ky, z): z in real
// space, x and y still transformed (kx < nx/2 in rows, nx/2 in nyq). The
// field is v(x, y, z) = C2R_x of sum_ky S e^{2 pi i ky y / ny}, so for the
// tensor-product stencil of a blob component (weights wx, wy, wz on the
// recorded nodes), J v = sum_z wz(z) Re sum_{kx, ky} c_kx Wx(kx) Wy(ky)
// S(kx, ky, z), with Wa(k) = sum_m wa[m] exp(+2 pi i k (base_a + m) / n_a)
// and c = 1 at kx = 0 and nx/2 (real there after the inverse), 2 between.
// J L v takes -(lam_x + lam_y) S + (S(z + 1) + S(z - 1) - 2 S(z)) / h^2 in
// place of S (the 7-point Laplacian: its x and y parts diagonal in kx, ky).
// One workgroup per (blob component, replica), a fixed-order reduction;
// then du and dp as in the step-4 gather.
template <typename T>
__global__ void __launch_bounds__(256) k_spec_gather(const RepDesc<T>* __restrict__ rd) {
    __shared__ double red[2][256];
    const RepDesc<T>& R = rd[blockIdx.y];
    const int o = (int)blockIdx.x;
    if (o >= 3 * R.bp.nb) return;
    const int bl = o / 3, a = o - 3 * bl;
    const GridDesc<T>& g = R.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz, H = nx / 2, W = H + 1;
    const gptr<const double> rec = as_global((const double*)R.bb.stc) + (long long)o * kStcPerComp;
    const int bx = (int)rec[0], by = (int)rec[1], bz = (int)rec[2];
    double wx[4], wy[4], wz[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        wx[m] = rec[3 + m];
        wy[m] = rec[7 + m];
        wz[m] = rec[11 + m];
    }
    const double ih2 = 1.0 / (g.h * g.h);
    const gptr<const cplx<T>> spec = as_global((const cplx<T>*)g.spec) + (long long)a * g.nspec;
    const gptr<const cplx<T>> nyq = as_global((const cplx<T>*)g.nyq) + (long long)a * nz * ny;
    const gptr<const cplx<T>> twx = as_global(g.twx), twy = as_global(g.twy);
    const gptr<const T> lx = as_global(g.lx), ly = as_global(g.ly);
    int zs[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        int z = bz - 1 + j;
        z %= nz;
        zs[j] = z < 0 ? z + nz : z;
    }
    double sv = 0.0, sl = 0.0;
    for (int idx = threadIdx.x; idx < W * ny; idx += blockDim.x) {
        const int ky = idx / W, kx = idx - ky * W;
        // Wx(kx) Wy(ky): the forward twiddles exp(-2 pi i j / n), conjugated
        double xr = 0, xi = 0, yr = 0, yi = 0;
        int ix = (int)(((long long)kx * bx) % nx), iy = (int)(((long long)ky * by) % ny);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const cplx<T> ex = twx[ix], ey = twy[iy];
            xr += wx[m] * (double)ex.x;
            xi -= wx[m] * (double)ex.y;
            yr += wy[m] * (double)ey.x;
            yi -= wy[m] * (double)ey.y;
            ix += kx;
            if (ix >= nx) ix -= nx;
            iy += ky;
            if (iy >= ny) iy -= ny;
        }
        const double cw = (kx == 0 || kx == H) ? 1.0 : 2.0;
        const double cr = cw * (xr * yr - xi * yi), ci = cw * (xr * yi + xi * yr);
        const double lam = (double)lx[kx] + (double)ly[ky];
        double sr[6], si[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const cplx<T> v = kx < H ? spec[((long long)zs[j] * ny + ky) * g.Wp + kx] : nyq[(long long)zs[j] * ny + ky];
            sr[j] = (double)v.x;
            si[j] = (double)v.y;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int j = m + 1;
            sv += wz[m] * (cr * sr[j] - ci * si[j]);
            const double lr = -lam * sr[j] + (sr[j + 1] + sr[j - 1] - 2.0 * sr[j]) * ih2;
            const double li = -lam * si[j] + (si[j + 1] + si[j - 1] - 2.0 * si[j]) * ih2;
            sl += wz[m] * (cr * lr - ci * li);
        }
    }
    red[0][threadIdx.x] = sv;
    red[1][threadIdx.x] = sl;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const BlobBufs& bb = R.bb;
        const BlobParams& bp = R.bp;
        const double J = red[0][0];
        bb.Jhvt[o] = J;
        bb.JLvt[o] = red[1][0];
        double du = 0.0;
        if (bp.slip == 2) du += bb.Jhvn[o] - bb.Jn[o];
        if (bp.slip >= 1) du += 0.5 * (bp.eta / bp.rho) * bp.dt * bb.lag[o];
        bb.du[o] = du;
        bb.dp[o] = bb.me[bl] * (bb.u[o] - J - du);
    }
}

// --------------------------------------------------------------- dispatch
// Plans: (E, R0, R1, R2) per (precision, N); a radix of 1 ends the list.
template <typename T, int N>
struct Plan {
    static constexpr bool ok = false;
};
#define ICM_PLAN(TT, NN, EE, A, B_, C)                 \
    template <>                                        \
    struct Plan<TT, NN> {                              \
        static constexpr bool ok = true;               \
        static constexpr int E = EE, R0 = A, R1 = B_, R2 = C; \
    };
ICM_PLAN(float, 16, 16, 16, 1, 1)
ICM_PLAN(float, 32, 16, 16, 2, 1)
ICM_PLAN(float, 48, 12, 4, 4, 3)
ICM_PLAN(float, 64, 16, 16, 4, 1)
ICM_PLAN(float, 128, 16, 16, 8, 1)
ICM_PLAN(float, 256, 16, 16, 16, 1)
ICM_PLAN(float, 512, 16, 8, 8, 8)
ICM_PLAN(double, 16, 8, 8, 2, 1)
ICM_PLAN(double, 32, 8, 8, 4, 1)
ICM_PLAN(double, 48, 12, 4, 4, 3)
ICM_PLAN(double, 64, 8, 8, 8, 1)
ICM_PLAN(double, 128, 8, 8, 8, 2)
ICM_PLAN(double, 256, 8, 8, 8, 4)
ICM_PLAN(double, 512, 8, 8, 8, 8)
#undef ICM_PLAN

// The z pass holds three components per thread; a smaller E keeps its
// register use (and so its occupancy) comparable to the other passes.
template <typename T, int N>
struct PlanZ : Plan<T, N> {};
#define ICM_PLANZ(TT, NN, EE, A, B_, C)                       \
    template <>                                               \
    struct PlanZ<TT, NN> {                                    \
        static constexpr bool ok = true;                      \
        static constexpr int E = EE, R0 = A, R1 = B_, R2 = C; \
    };
// FP32: eight values per thread halve the registers of the three-component
// pencil (one more LDS exchange per transform), which doubles the waves the
// pass keeps in flight; measured faster at 256^3.
ICM_PLANZ(float, 64, 8, 8, 8, 1)
ICM_PLANZ(float, 128, 8, 8, 4, 4)
ICM_PLANZ(float, 256, 8, 8, 8, 4)
ICM_PLANZ(float, 512, 8, 8, 8, 8)
#undef ICM_PLANZ

// Kernels whose LDS exceeds 64 KB opt in to the larger gfx950 allocation.
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

template <typename T>
int pairs_per_block(int N, int TL, int xt) {
    int P = (xt > 0 ? xt : 256) / TL;
    if (P < 1) P = 1;
    while (P > 1 && ((size_t)N + (size_t)P * (N + N / 16 + 1)) * sizeof(cplx<T>) > kLdsMax) P /= 2;
    return P;
}

template <typename T, int N>
bool y_fast(const Batch<T>& Bt, int dir, hipStream_t s) {
    using Pl = Plan<T, N>;
    if constexpr (!Pl::ok) {
        return false;
    } else {
        const GridDesc<T>& g = Bt.g;
        constexpr int TL = N / Pl::E;
        int B = g.By;
        while (B > 1 && B * TL > 512) B /= 2;
        const dim3 grid((unsigned)((g.nx / 2 + B - 1) / B + 1), g.nz, 3 * Bt.nrep);
        const size_t lds = (size_t)N * (B + 1) * sizeof(cplx<T>);
        if (dir < 0) {
            allow_lds(k_y_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, -1>, lds);
            hipLaunchKernelGGL((k_y_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, -1>), grid, dim3(B * TL), lds, s, Bt.d,
                               B);
        } else {
            allow_lds(k_y_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, 1>, lds);
            hipLaunchKernelGGL((k_y_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, 1>), grid, dim3(B * TL), lds, s, Bt.d,
                               B);
        }
        return true;
    }
}

template <typename T, int N, typename Pl, int SRC = 0>
bool z_fast_plan(const Batch<T>& Bt, int solve, bool project, hipStream_t s, bool carry) {
    if constexpr (!Pl::ok) {
        return false;
    } else {
        const GridDesc<T>& g = Bt.g;
        constexpr int TL = N / Pl::E;
        int B = g.Bz;
        while (B > 1 && B * TL > 512) B /= 2;
        const dim3 grid((unsigned)((g.nx / 2 + B - 1) / B + 1), g.ny, Bt.nrep);
        // twiddles, exchange buffer, d_z and the z eigenvalues
        const size_t lds = (size_t)N * (B + 2) * sizeof(cplx<T>) + (size_t)N * sizeof(T);
        allow_lds(k_z_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, SRC>, lds);
        hipLaunchKernelGGL((k_z_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2, SRC>), grid, dim3(B * TL), lds, s, Bt.d,
                           B, solve, (project ? 1 : 0) | (carry ? 2 : 0));
        return true;
    }
}

template <typename T, int N>
bool z_fast(const Batch<T>& Bt, int solve, bool project, hipStream_t s, bool carry) {
    if (Bt.g.zsmall) return z_fast_plan<T, N, PlanZ<T, N>>(Bt, solve, project, s, carry);
    return z_fast_plan<T, N, Plan<T, N>>(Bt, solve, project, s, carry);
}

template <typename T, int N>
bool z_fast_src(const Batch<T>& Bt, int solve, hipStream_t s, bool carry, bool acc) {
    if (acc) {
        if (Bt.g.zsmall) return z_fast_plan<T, N, PlanZ<T, N>, 2>(Bt, solve, true, s, carry);
        return z_fast_plan<T, N, Plan<T, N>, 2>(Bt, solve, true, s, carry);
    }
    if (Bt.g.zsmall) return z_fast_plan<T, N, PlanZ<T, N>, 1>(Bt, solve, true, s, carry);
    return z_fast_plan<T, N, Plan<T, N>, 1>(Bt, solve, true, s, carry);
}

template <typename T, int N>
bool xf_fast(const Batch<T>& Bt, int in, hipStream_t s) {
    using Pl = Plan<T, N>;
    if constexpr (!Pl::ok) {
        return false;
    } else {
        const GridDesc<T>& g = Bt.g;
        constexpr int TL = N / Pl::E;
        const int P = pairs_per_block<T>(N, TL, g.xt);
        const long long npairs = (long long)g.ny * g.nz / 2;
        const dim3 grid((unsigned)((npairs + P - 1) / P), 3 * Bt.nrep);
        const size_t lds = (size_t)(N + P * xline<N>()) * sizeof(cplx<T>);
        hipLaunchKernelGGL((k_xfwd_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2>), grid, dim3(P * TL), lds, s, Bt.d, in,
                           P);
        return true;
    }
}

template <typename T, int N>
bool xi_fast(const Batch<T>& Bt, int out, int acc, hipStream_t s) {
    using Pl = Plan<T, N>;
    if constexpr (!Pl::ok) {
        return false;
    } else {
        const GridDesc<T>& g = Bt.g;
        constexpr int TL = N / Pl::E;
        const int P = pairs_per_block<T>(N, TL, g.xt);
        const long long npairs = (long long)g.ny * g.nz / 2;
        const dim3 grid((unsigned)((npairs + P - 1) / P), 3 * Bt.nrep);
        const size_t lds = (size_t)(N + P * xline<N>()) * sizeof(cplx<T>);
        hipLaunchKernelGGL((k_xinv_fast<T, N, Pl::E, Pl::R0, Pl::R1, Pl::R2>), grid, dim3(P * TL), lds, s, Bt.d, out,
                           P, acc);
        return true;
    }
}

#define ICM_SWITCH_N(n, CALL) \
    switch (n) {              \
        case 16: return CALL(16); \
        case 32: return CALL(32); \
        case 48: return CALL(48); \
        case 64: return CALL(64); \
        case 128: return CALL(128); \
        case 256: return CALL(256); \
        case 512: return CALL(512); \
        default: return false;    \
    }

}  // namespace

template <typename T>
bool fast_fft_available(int nx, int ny, int nz) {
    auto has = [](int n) {
        switch (n) {
            case 16: return Plan<T, 16>::ok;
            case 32: return Plan<T, 32>::ok;
            case 48: return Plan<T, 48>::ok;
            case 64: return Plan<T, 64>::ok;
            case 128: return Plan<T, 128>::ok;
            case 256: return Plan<T, 256>::ok;
            case 512: return Plan<T, 512>::ok;
            default: return false;
        }
    };
    return has(nx) && has(ny) && has(nz);
}

template <typename T>
bool fast_fft_y(const Batch<T>& B, int dir, hipStream_t s) {
#define C(NN) y_fast<T, NN>(B, dir, s)
    ICM_SWITCH_N(B.g.ny, C)
#undef C
}
template <typename T>
bool fast_fft_z_solve(const Batch<T>& B, int solve, bool project, hipStream_t s, bool carry) {
#define C(NN) z_fast<T, NN>(B, solve, project, s, carry)
    ICM_SWITCH_N(B.g.nz, C)
#undef C
}
template <typename T>
void launch_spectral_gather(const Batch<T>& B, hipStream_t s) {
    if (B.max_nb > 0) hipLaunchKernelGGL(k_spec_gather<T>, dim3(3 * B.max_nb, B.nrep), dim3(256), 0, s, B.d);
}
template <typename T>
bool fast_fft_z_solve_from_blobs(const Batch<T>& B, int solve, hipStream_t s, bool carry, bool accumulate) {
    if (!B.g.fast) return false;
#define C(NN) z_fast_src<T, NN>(B, solve, s, carry, accumulate)
    ICM_SWITCH_N(B.g.nz, C)
#undef C
}
template <typename T>
bool fast_fft_x_forward(const Batch<T>& B, int in, hipStream_t s) {
#define C(NN) xf_fast<T, NN>(B, in, s)
    ICM_SWITCH_N(B.g.nx, C)
#undef C
}
template <typename T>
bool fast_fft_x_inverse(const Batch<T>& B, int out, int acc, hipStream_t s) {
#define C(NN) xi_fast<T, NN>(B, out, acc, s)
    ICM_SWITCH_N(B.g.nx, C)
#undef C
}

#define ICM_INST(T)                                                                \
    template bool fast_fft_available<T>(int, int, int);                            \
    template bool fast_fft_y<T>(const Batch<T>&, int, hipStream_t);                \
    template bool fast_fft_z_solve<T>(const Batch<T>&, int, bool, hipStream_t, bool); \
    template bool fast_fft_z_solve_from_blobs<T>(const Batch<T>&, int, hipStream_t, bool, bool); \
    template void launch_spectral_gather<T>(const Batch<T>&, hipStream_t); \
    template bool fast_fft_x_forward<T>(const Batch<T>&, int, hipStream_t);        \
    template bool fast_fft_x_inverse<T>(const Batch<T>&, int, int, hipStream_t);
ICM_INST(float)
ICM_INST(double)
#undef ICM_INST

}  // namespace icm
