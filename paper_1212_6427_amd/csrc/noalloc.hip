// icm_solve_noalloc: the FFT-diagonalised Helmholtz solve with projection of
// Sec. III.D on caller-owned device fields, with every intermediate buffer
// (descriptor, twiddle and symbol tables, spectrum) in one file-scope device
// array, so that the call allocates no device memory.
//
// The array is `scratch`. On the host its name is only a stand-in for the
// symbol: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept in g_scratch, and only that address is handed to kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/icm.h"
#include "icm_internal.h"

namespace icm {
icm_status fail_without_context(icm_status st, const char* fmt, ...);
}

namespace {

using icm::cplx;

// The largest scratch need is the spectrum: 3 x nz x ny rows of (about)
// nx/2 complex values. 64 MiB holds it for 128^3 in FP64 and about 4.5 M
// cells in FP32.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<unsigned char*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of this device's scratch array (set up on first use).
icm_status scratch_of_current_device(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return icm::fail_without_context(ICM_E_DEVICE, "icm_solve_noalloc: hipGetDevice failed: %s",
                                         hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return icm::fail_without_context(ICM_E_UNSUPPORTED, "icm_solve_noalloc: device %d beyond the first %d", dev,
                                         kMaxDevices);
    unsigned char* p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            void* addr = nullptr;
            e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !addr)
                return icm::fail_without_context(ICM_E_DEVICE,
                                                 "icm_solve_noalloc: hipGetSymbolAddress(scratch) failed: %s",
                                                 hipGetErrorString(e));
            p = static_cast<unsigned char*>(addr);
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return ICM_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Carve the solve's buffers from the scratch base (base == nullptr: sizing).
template <typename T>
size_t carve(unsigned char* base, icm::GridDesc<T>& g, icm::RepDesc<T>** desc) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = align256(off);
        unsigned char* r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    *desc = reinterpret_cast<icm::RepDesc<T>*>(take(sizeof(icm::RepDesc<T>)));
    g.spec = reinterpret_cast<cplx<T>*>(take(3 * (size_t)g.nspec * sizeof(cplx<T>)));
    g.nyq = g.fast ? reinterpret_cast<cplx<T>*>(take(3 * (size_t)g.nz * g.ny * sizeof(cplx<T>))) : nullptr;
    g.twx = reinterpret_cast<cplx<T>*>(take(g.nx * sizeof(cplx<T>)));
    g.twy = reinterpret_cast<cplx<T>*>(take(g.ny * sizeof(cplx<T>)));
    g.twz = reinterpret_cast<cplx<T>*>(take(g.nz * sizeof(cplx<T>)));
    g.dx_hat = reinterpret_cast<cplx<T>*>(take(g.W * sizeof(cplx<T>)));
    g.dy_hat = reinterpret_cast<cplx<T>*>(take(g.ny * sizeof(cplx<T>)));
    g.dz_hat = reinterpret_cast<cplx<T>*>(take(g.nz * sizeof(cplx<T>)));
    g.lx = reinterpret_cast<T*>(take(g.W * sizeof(T)));
    g.ly = reinterpret_cast<T*>(take(g.ny * sizeof(T)));
    g.lz = reinterpret_cast<T*>(take(g.nz * sizeof(T)));
    return align256(off);
}

// Twiddles exp(-2 pi i m / N) and the difference symbols of each axis:
// Dhat = (e^{i theta} - 1)/h = (-2 sin^2(theta/2) + i sin theta)/h and
// lambda = 4 sin^2(theta/2)/h^2, theta = 2 pi m / N, evaluated in FP64 with
// sinpi / cospi and rounded to T.
template <typename T>
__device__ void axis_tables(int m, int n, int nsym, double h, cplx<T>* tw, cplx<T>* d, T* l) {
    if (m < n) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = cplx<T>{(T)c, (T)(-s)};
    }
    if (m < nsym) {
        const double s2 = sinpi((double)m / (double)n);
        const double st = sinpi(2.0 * (double)m / (double)n);
        d[m] = cplx<T>{(T)(-2.0 * s2 * s2 / h), (T)(st / h)};
        l[m] = (T)(4.0 * s2 * s2 / (h * h));
    }
}

template <typename T>
__global__ void k_noalloc_setup(icm::RepDesc<T> desc, icm::RepDesc<T>* dst) {
    const icm::GridDesc<T>& g = desc.g;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m == 0) *dst = desc;
    axis_tables<T>(m, g.nx, g.W, g.h, const_cast<cplx<T>*>(g.twx), const_cast<cplx<T>*>(g.dx_hat),
                   const_cast<T*>(g.lx));
    axis_tables<T>(m, g.ny, g.ny, g.h, const_cast<cplx<T>*>(g.twy), const_cast<cplx<T>*>(g.dy_hat),
                   const_cast<T*>(g.ly));
    axis_tables<T>(m, g.nz, g.nz, g.h, const_cast<cplx<T>*>(g.twz), const_cast<cplx<T>*>(g.dz_hat),
                   const_cast<T*>(g.lz));
}

template <typename T>
icm_status solve_t(const int32_t n[3], double h, double a, double b, const void* rhs, void* out, hipStream_t s,
                   unsigned char* base) {
    icm::GridDesc<T> g{};
    icm::grid_shape(g, n, h);
    icm::RepDesc<T>* ddesc = nullptr;
    const size_t need = carve<T>(nullptr, g, &ddesc);
    if (need > kScratchBytes)
        return icm::fail_without_context(ICM_E_INVALID,
                                         "icm_solve_noalloc: a %d x %d x %d grid in %s needs %zu bytes of scratch, "
                                         "more than the %zu the library holds",
                                         n[0], n[1], n[2], sizeof(T) == 8 ? "FP64" : "FP32", need, kScratchBytes);
    carve<T>(base, g, &ddesc);
    g.rhs = static_cast<T*>(const_cast<void*>(rhs));
    g.v = static_cast<T*>(out);
    icm::RepDesc<T> d{};
    d.g = g;
    d.solve[icm::kSolveH1] = icm::SolveCoef{a, b, 1.0 / (double)g.ncell};
    const int m = std::max(g.nx, std::max(g.ny, g.nz));
    hipLaunchKernelGGL(k_noalloc_setup<T>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, d, ddesc);
    icm::Batch<T> B{};
    B.d = ddesc;
    B.nrep = 1;
    B.g = g;
    B.kernel = 3;
    B.max_nb = 0;
    B.one = nullptr;
    icm::launch_fft_x_forward(B, icm::kFieldRhs, s);
    icm::launch_fft_y(B, -1, s);
    icm::launch_fft_z_solve(B, icm::kSolveH1, true, s);
    icm::launch_fft_y(B, 1, s);
    icm::launch_fft_x_inverse(B, icm::kFieldV, false, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return icm::fail_without_context(ICM_E_DEVICE, "icm_solve_noalloc: launch failed: %s", hipGetErrorString(e));
    return ICM_OK;
}

}  // namespace

extern "C" icm_status icm_solve_noalloc(const int32_t n[3], double h, double a, double b, int32_t precision,
                                        const void* rhs, void* out, void* stream) {
    if (!n || !rhs || !out) return icm::fail_without_context(ICM_E_INVALID, "icm_solve_noalloc: NULL argument");
    for (int ax = 0; ax < 3; ++ax) {
        icm::FFTPlan pl;
        if (n[ax] < 4 || n[ax] > 512 || (n[ax] & 1) || !icm::factor_plan(n[ax], pl))
            return icm::fail_without_context(
                ICM_E_INVALID, "icm_solve_noalloc: N[%d] = %d must be even, in [4, 512], with prime factors 2 and 3 only",
                ax, n[ax]);
    }
    if (!(h > 0) || !(a > 0) || !(b >= 0) || !std::isfinite(h) || !std::isfinite(a) || !std::isfinite(b))
        return icm::fail_without_context(ICM_E_INVALID, "icm_solve_noalloc: need h > 0, a > 0 and b >= 0 (finite)");
    if (precision != ICM_FP64 && precision != ICM_FP32_GRID)
        return icm::fail_without_context(ICM_E_INVALID, "icm_solve_noalloc: precision must be ICM_FP64 or "
                                                        "ICM_FP32_GRID");
    unsigned char* base = nullptr;
    const icm_status st = scratch_of_current_device(&base);
    if (st != ICM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return precision == ICM_FP64 ? solve_t<double>(n, h, a, b, rhs, out, s, base)
                                 : solve_t<float>(n, h, a, b, rhs, out, s, base);
}
