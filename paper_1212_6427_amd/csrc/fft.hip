// Batched 3-D real FFTs with the spectral Helmholtz solve and projection of
// Sec. III.D: "solve the velocity equation without the pressure gradient by
// diagonalising the discrete Laplacian with a Fourier transform, then project
// onto discretely divergence-free fields".
//
// Passes (all hand-written, mixed-radix 2/3/4/8 Stockham in LDS):
//   x forward : real rows -> half spectrum, two real rows packed into one
//               complex row and separated by Hermitian symmetry;
//   y forward : complex columns, in place;
//   z + solve : the three components of a (kx, ky) pencil are transformed
//               along z, multiplied per mode by P-hat / (a + b lambda), and
//               transformed back, in one kernel (P-hat couples components);
//   y inverse, x inverse (complex -> real rows, optionally accumulated).
#include "icm_internal.h"

namespace icm {

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsBudget = 64 * 1024;

// ------------------------------------------------------------- butterflies
template <typename T, int DIR>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft3(cplx<T>* v) {
    // X1 = t + DIR i (sqrt3/2) d, X2 = t - DIR i (sqrt3/2) d with
    // s = v1 + v2, d = v1 - v2, t = v0 - s/2 (w = exp(DIR 2 pi i / 3)).
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
__device__ __forceinline__ void dft4(cplx<T>* v) {
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
__device__ __forceinline__ void dft8(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, DIR>(e);
    dft4<T, DIR>(o);
    const T r = (T)0.70710678118654752440;
    // o[m] *= exp(DIR 2 pi i m / 8)
    o[1] = {r * (o[1].x - DIR * o[1].y), r * (o[1].y + DIR * o[1].x)};
    o[2] = cmul_i(o[2], DIR);
    o[3] = {r * (-o[3].x - DIR * o[3].y), r * (-o[3].y + DIR * o[3].x)};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v[m] = cadd(e[m], o[m]);
        v[m + 4] = csub(e[m], o[m]);
    }
}

// One Stockham stage of radix R over nlines lines. Element n of line l is at
// base[l * ls + n * es]. Ns is the product of the radices already applied.
template <typename T, int R, int DIR>
__device__ __forceinline__ void stage(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                      int N, int Ns, int nlines, int ls, int es,
                                      const cplx<T>* __restrict__ tw) {
    const int nbf = N / R;
    const int total = nbf * nlines;
    const int twstep = N / (Ns * R);
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int line = t / nbf;
        const int j = t - line * nbf;
        const int k = j % Ns;
        const cplx<T>* s = src + line * ls;
        cplx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cplx<T> x = s[(j + r * nbf) * es];
            if (r > 0) {
                cplx<T> w = tw[r * k * twstep];
                if (DIR > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            v[r] = x;
        }
        if (R == 2) dft2<T, DIR>(v);
        if (R == 3) dft3<T, DIR>(v);
        if (R == 4) dft4<T, DIR>(v);
        if (R == 8) dft8<T, DIR>(v);
        const int base = (j / Ns) * Ns * R + k;
        cplx<T>* d = dst + line * ls;
#pragma unroll
        for (int r = 0; r < R; ++r) d[(base + r * Ns) * es] = v[r];
    }
}

// Full transform of nlines lines; returns the buffer holding the result.
template <typename T, int DIR>
__device__ cplx<T>* lds_fft(cplx<T>* a, cplx<T>* b, const FFTPlan& pl, int nlines, int ls, int es,
                            const cplx<T>* tw) {
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.radix[st];
        if (R == 2) stage<T, 2, DIR>(a, b, pl.n, Ns, nlines, ls, es, tw);
        else if (R == 3) stage<T, 3, DIR>(a, b, pl.n, Ns, nlines, ls, es, tw);
        else if (R == 4) stage<T, 4, DIR>(a, b, pl.n, Ns, nlines, ls, es, tw);
        else stage<T, 8, DIR>(a, b, pl.n, Ns, nlines, ls, es, tw);
        __syncthreads();
        cplx<T>* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// ----------------------------------------------------------------- x pass
// Rows 2p and 2p+1 of a component (same z, y and y+1) form z = a + i b.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_xfwd(const RepDesc<T>* __restrict__ rd, int in_sel, int pp) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
    const GridDesc<T>& g = rd[blockIdx.y / 3].g;
    const T* __restrict__ in = field_of(g, in_sel);
    const int N = g.nx, W = g.W;
    cplx<T>* tw = sm;
    cplx<T>* b0 = sm + N;
    cplx<T>* b1 = b0 + pp * N;
    const int c = (int)(blockIdx.y % 3);
    const long long npairs = (long long)g.ny * g.nz / 2;
    const long long p0 = (long long)blockIdx.x * pp;
    load_twiddles(tw, g.twx, N);
    const T* src = in + (long long)c * g.ncell;
    for (int idx = threadIdx.x; idx < pp * N; idx += blockDim.x) {
        const int l = idx / N, x = idx - l * N;
        const long long p = p0 + l;
        cplx<T> z = {0, 0};
        if (p < npairs) z = {src[(2 * p) * N + x], src[(2 * p + 1) * N + x]};
        b0[idx] = z;
    }
    __syncthreads();
    cplx<T>* r = lds_fft<T, -1>(b0, b1, g.px, pp, N, 1, tw);
    cplx<T>* dst = g.spec + (long long)c * g.nspec;
    for (int idx = threadIdx.x; idx < pp * W; idx += blockDim.x) {
        const int l = idx / W, k = idx - l * W;
        const long long p = p0 + l;
        if (p >= npairs) continue;
        const cplx<T> zk = r[l * N + k];
        const cplx<T> zc = cconj(r[l * N + ((N - k) % N)]);
        const cplx<T> s = cadd(zk, zc), d = csub(zk, zc);
        dst[(2 * p) * g.Wp + k] = {(T)0.5 * s.x, (T)0.5 * s.y};
        dst[(2 * p + 1) * g.Wp + k] = {(T)0.5 * d.y, (T)-0.5 * d.x};
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_xinv(const RepDesc<T>* __restrict__ rd, int out_sel, int pp,
                                                   int accumulate) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
    const GridDesc<T>& g = rd[blockIdx.y / 3].g;
    T* __restrict__ out = field_of(g, out_sel);
    const int N = g.nx, W = g.W, H = g.nx / 2;
    cplx<T>* tw = sm;
    cplx<T>* b0 = sm + N;
    cplx<T>* b1 = b0 + pp * N;
    const int c = (int)(blockIdx.y % 3);
    const long long npairs = (long long)g.ny * g.nz / 2;
    const long long p0 = (long long)blockIdx.x * pp;
    load_twiddles(tw, g.twx, N);
    const cplx<T>* src = g.spec + (long long)c * g.nspec;
    for (int idx = threadIdx.x; idx < pp * N; idx += blockDim.x) {
        const int l = idx / N, k = idx - l * N;
        const long long p = p0 + l;
        cplx<T> z = {0, 0};
        if (p < npairs) {
            cplx<T> A, B;
            if (k <= H) {
                A = src[(2 * p) * g.Wp + k];
                B = src[(2 * p + 1) * g.Wp + k];
                if (k == 0 || k == H) {
                    A.y = 0;
                    B.y = 0;
                }
            } else {
                A = cconj(src[(2 * p) * g.Wp + (N - k)]);
                B = cconj(src[(2 * p + 1) * g.Wp + (N - k)]);
            }
            z = {A.x - B.y, A.y + B.x};
        }
        b0[idx] = z;
    }
    __syncthreads();
    cplx<T>* r = lds_fft<T, 1>(b0, b1, g.px, pp, N, 1, tw);
    T* dst = out + (long long)c * g.ncell;
    T* vv = g.v + (long long)c * g.ncell;
    for (int idx = threadIdx.x; idx < pp * N; idx += blockDim.x) {
        const int l = idx / N, x = idx - l * N;
        const long long p = p0 + l;
        if (p >= npairs) continue;
        const cplx<T> z = r[idx];
        if (accumulate == kXinvAlsoV) {
            dst[(2 * p) * N + x] = z.x;
            dst[(2 * p + 1) * N + x] = z.y;
            vv[(2 * p) * N + x] += z.x;
            vv[(2 * p + 1) * N + x] += z.y;
        } else if (accumulate) {
            dst[(2 * p) * N + x] += z.x;
            dst[(2 * p + 1) * N + x] += z.y;
        } else {
            dst[(2 * p) * N + x] = z.x;
            dst[(2 * p + 1) * N + x] = z.y;
        }
    }
}

// ----------------------------------------------------------------- y pass
template <typename T, int DIR>
__global__ void __launch_bounds__(kThreads) k_ypass(const RepDesc<T>* __restrict__ rd, int B) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
    const GridDesc<T>& g = rd[blockIdx.z / 3].g;
    const int N = g.ny, W = g.W;
    cplx<T>* tw = sm;
    cplx<T>* b0 = sm + N;
    cplx<T>* b1 = b0 + N * B;
    const int kx0 = blockIdx.x * B;
    const int bw = min(B, W - kx0);
    const int z = blockIdx.y;
    const int c = (int)(blockIdx.z % 3);
    load_twiddles(tw, g.twy, N);
    cplx<T>* base = g.spec + (long long)c * g.nspec + (long long)z * N * g.Wp + kx0;
    for (int idx = threadIdx.x; idx < N * B; idx += blockDim.x) {
        const int y = idx / B, b = idx - y * B;
        b0[idx] = (b < bw) ? base[(long long)y * g.Wp + b] : cplx<T>{0, 0};
    }
    __syncthreads();
    cplx<T>* r = lds_fft<T, DIR>(b0, b1, g.py, B, 1, B, tw);
    for (int idx = threadIdx.x; idx < N * B; idx += blockDim.x) {
        const int y = idx / B, b = idx - y * B;
        if (b < bw) base[(long long)y * g.Wp + b] = r[idx];
    }
}

// -------------------------------------------------------- z pass + solve
template <typename T>
__global__ void __launch_bounds__(kThreads) k_zsolve(const RepDesc<T>* __restrict__ rd, int B, int solve,
                                                     int project) {
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_raw);
    const GridDesc<T>& g = rd[blockIdx.z].g;
    const SolveCoef sc = rd[blockIdx.z].solve[solve];
    const int N = g.nz, W = g.W, NY = g.ny;
    const int L3 = 3 * B;
    cplx<T>* tw = sm;
    cplx<T>* b0 = sm + N;
    cplx<T>* b1 = b0 + N * L3;
    const int kx0 = blockIdx.x * B;
    const int bw = min(B, W - kx0);
    const int y = blockIdx.y;
    load_twiddles(tw, g.twz, N);
    // element (z, c, b) at z * 3B + c * B + b
    for (int idx = threadIdx.x; idx < N * L3; idx += blockDim.x) {
        const int z = idx / L3, rem = idx - z * L3;
        const int c = rem / B, b = rem - c * B;
        b0[idx] = (b < bw) ? g.spec[(long long)c * g.nspec + ((long long)z * NY + y) * g.Wp + kx0 + b]
                           : cplx<T>{0, 0};
    }
    __syncthreads();
    cplx<T>* r = lds_fft<T, -1>(b0, b1, g.pz, L3, 1, L3, tw);
    cplx<T>* o = (r == b0) ? b1 : b0;
    const T ly = g.ly[y];
    const cplx<T> dy = g.dy_hat[y];
    for (int idx = threadIdx.x; idx < N * B; idx += blockDim.x) {
        const int z = idx / B, b = idx - z * B;
        if (b >= bw) continue;
        const int kx = kx0 + b;
        cplx<T>* e = r + z * L3 + b;
        cplx<T> w0 = e[0], w1 = e[B], w2 = e[2 * B];
        const T lam = g.lx[kx] + ly + g.lz[z];
        const T f = (T)(sc.scale / (sc.a + sc.b * (double)lam));
        w0 = {w0.x * f, w0.y * f};
        w1 = {w1.x * f, w1.y * f};
        w2 = {w2.x * f, w2.y * f};
        if ((project & 1) && lam > (T)0) {
            const cplx<T> dx = g.dx_hat[kx], dz = g.dz_hat[z];
            const cplx<T> d = cadd(cadd(cmul(dx, w0), cmul(dy, w1)), cmul(dz, w2));
            const T il = (T)1 / lam;
            const cplx<T> dd = {d.x * il, d.y * il};
            w0 = csub(w0, cmul(cconj(dx), dd));
            w1 = csub(w1, cmul(cconj(dy), dd));
            w2 = csub(w2, cmul(cconj(dz), dd));
        }
        if ((project & 2) && g.k0 && kx == 0 && y == 0 && z == 0) carry_mean_mode(rd[blockIdx.z], solve, w0, w1, w2);
        e[0] = w0;
        e[B] = w1;
        e[2 * B] = w2;
    }
    __syncthreads();
    cplx<T>* r2 = lds_fft<T, 1>(r, o, g.pz, L3, 1, L3, tw);
    for (int idx = threadIdx.x; idx < N * L3; idx += blockDim.x) {
        const int z = idx / L3, rem = idx - z * L3;
        const int c = rem / B, b = rem - c * B;
        if (b < bw) g.spec[(long long)c * g.nspec + ((long long)z * NY + y) * g.Wp + kx0 + b] = r2[idx];
    }
}

int pow2_floor(long long x) {
    int p = 1;
    while ((long long)p * 2 <= x) p *= 2;
    return p;
}

}  // namespace

namespace {
size_t xpass_lines(int N, size_t cs) {
    long long pp = (long long)(kLdsBudget / cs - N) / (2 * N);
    return (size_t)(pp < 1 ? 1 : (pp > 16 ? 16 : pp));
}
int ypass_width(int N, size_t cs) {
    long long b = (long long)(kLdsBudget / cs - N) / (2 * N);
    return pow2_floor(b < 1 ? 1 : (b > 16 ? 16 : b));
}
int zpass_width(int N, size_t cs) {
    long long b = (long long)(kLdsBudget / cs - N) / (6 * N);
    return pow2_floor(b < 1 ? 1 : (b > 16 ? 16 : b));
}
}  // namespace

template <typename T>
void launch_fft_x_forward(const Batch<T>& B, int in, hipStream_t s) {
    const GridDesc<T>& g = B.g;
    if (g.fast && fast_fft_x_forward(B, in, s)) return;
    const size_t cs = sizeof(cplx<T>);
    const int N = g.nx;
    const long long pp = (long long)xpass_lines(N, cs);
    const long long npairs = (long long)g.ny * g.nz / 2;
    const dim3 grid((unsigned)((npairs + pp - 1) / pp), 3 * B.nrep);
    const size_t lds = (size_t)(N + 2 * pp * N) * cs;
    hipLaunchKernelGGL(k_xfwd<T>, grid, dim3(kThreads), lds, s, B.d, in, (int)pp);
}

template <typename T>
void launch_fft_y(const Batch<T>& B, int dir, hipStream_t s) {
    const GridDesc<T>& g = B.g;
    if (g.fast && fast_fft_y(B, dir, s)) return;
    const size_t cs = sizeof(cplx<T>);
    const int N = g.ny;
    const int By = ypass_width(N, cs);
    const dim3 grid((unsigned)((g.W + By - 1) / By), g.nz, 3 * B.nrep);
    const size_t lds = (size_t)(N + 2 * N * By) * cs;
    if (dir < 0)
        hipLaunchKernelGGL((k_ypass<T, -1>), grid, dim3(kThreads), lds, s, B.d, By);
    else
        hipLaunchKernelGGL((k_ypass<T, 1>), grid, dim3(kThreads), lds, s, B.d, By);
}

template <typename T>
void launch_fft_z_solve(const Batch<T>& B, int solve, bool project, hipStream_t s, bool carry) {
    const GridDesc<T>& g = B.g;
    if (g.fast && fast_fft_z_solve(B, solve, project, s, carry)) return;
    const size_t cs = sizeof(cplx<T>);
    const int N = g.nz;
    const int Bz = zpass_width(N, cs);
    const dim3 grid((unsigned)((g.W + Bz - 1) / Bz), g.ny, B.nrep);
    const size_t lds = (size_t)(N + 6 * N * Bz) * cs;
    hipLaunchKernelGGL(k_zsolve<T>, grid, dim3(kThreads), lds, s, B.d, Bz, solve, (project ? 1 : 0) | (carry ? 2 : 0));
}

template <typename T>
void launch_fft_x_inverse(const Batch<T>& B, int out, int accumulate, hipStream_t s) {
    const GridDesc<T>& g = B.g;
    if (g.fast && fast_fft_x_inverse(B, out, accumulate, s)) return;
    const size_t cs = sizeof(cplx<T>);
    const int N = g.nx;
    const long long pp = (long long)xpass_lines(N, cs);
    const long long npairs = (long long)g.ny * g.nz / 2;
    const dim3 grid((unsigned)((npairs + pp - 1) / pp), 3 * B.nrep);
    const size_t lds = (size_t)(N + 2 * pp * N) * cs;
    hipLaunchKernelGGL(k_xinv<T>, grid, dim3(kThreads), lds, s, B.d, out, (int)pp, accumulate);
}

#define ICM_INST(T)                                                                     \
    template void launch_fft_x_forward<T>(const Batch<T>&, int, hipStream_t);           \
    template void launch_fft_y<T>(const Batch<T>&, int, hipStream_t);                   \
    template void launch_fft_z_solve<T>(const Batch<T>&, int, bool, hipStream_t, bool); \
    template void launch_fft_x_inverse<T>(const Batch<T>&, int, int, hipStream_t);
ICM_INST(float)
ICM_INST(double)
#undef ICM_INST

}  // namespace icm
