// Internal interfaces between the ICM context (api.hip) and the kernel
// launchers (fft.hip, grid.hip, blobs.hip). Everything here works on raw
// device pointers and one HIP stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "icm_common.h"

namespace icm {

constexpr int kMaxStages = 16;

// Mixed-radix (2, 3, 4, 8) Stockham plan of one FFT length.
struct FFTPlan {
    int n;
    int nst;
    int radix[kMaxStages];
};

// Field buffers of one replica. Real face fields hold 3 components of
// ncell values (x fastest); the spectrum holds 3 components of
// nz * ny rows of W = nx/2 + 1 complex values (kx fastest) at row pitch Wp.
template <typename T>
struct GridDesc {
    int nx, ny, nz, W;
    int Wp;            // spectrum row pitch (>= W, a multiple of 128 bytes)
    int fast;          // 1: register-resident FFT passes (all three N supported)
    int By, Bz;        // kx columns per block of the fast y and z passes
    long long ncell;   // nx * ny * nz
    long long nspec;   // nz * ny * Wp
    double h;
    T* v;              // fluid velocity v^n / v^{n+1}
    T* rhs;            // right-hand side / spread scratch field
    T* aux;            // inertial-correction field (dv~, dv)
    cplx<T>* spec;     // spectral work buffer
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
};

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
    double body[3];
    NoiseKey key;
};

// Blobs spread inside the right-hand-side kernel. stc holds, per blob and
// component a, the wrapped base nodes (as doubles) of the P-tap stencil on
// the a-component grid, the P weights of each axis, and the P derivative
// weights phi'(d)/h along axis a (kStcPerComp values per component).
// Blobs are binned by z-chunk of kRhsZChunk planes: chunk_count[c] blobs of
// chunk c are listed at chunk_list[c * cap]. A tile that meets more than
// kRhsTileCap blobs appends the excess (blob, tile) pairs to the overflow
// list, which launch_spread_overflow spreads with atomics.
constexpr int kRhsZChunk = 16;
constexpr int kRhsTileCap = 128;
constexpr int kStcPerComp = 3 + 4 * 4;
struct RhsBlobs {
    int nb;
    int kernel;
    int cap;                 // list capacity per chunk (>= nb)
    const double* stc;       // nb * 3 * kStcPerComp
    const double* F;         // nb * 3 forces (spread with S)
    const double* cdrift;    // nb drift coefficients kT m~_f / m~ (NULL = no drift)
    const int* chunk_count;  // n_chunks
    const int* chunk_list;   // n_chunks * cap
    int* ovf_count;          // 1
    int* ovf_list;           // 2 * ovf_cap ints (blob, tile)
    int ovf_cap;
};

// ------------------------------------------------------------------- FFT
// The x and y passes work on one component c (0..2) per launch, or on all
// three with c = -1.
template <typename T>
void launch_fft_x_forward(const GridDesc<T>& g, const T* in, hipStream_t s, int c = -1);
template <typename T>
void launch_fft_y(const GridDesc<T>& g, int dir, hipStream_t s, int c = -1);
template <typename T>
void launch_fft_z_solve(const GridDesc<T>& g, SolveCoef sc, bool project, hipStream_t s);
template <typename T>
void launch_fft_x_inverse(const GridDesc<T>& g, T* out, bool accumulate, hipStream_t s, int c = -1);
template <typename T>
void launch_fft_forward_solve_inverse(const GridDesc<T>& g, const T* in, T* out, bool accumulate,
                                      SolveCoef sc, bool project, hipStream_t s);

// Register-resident passes for N in {16, 32, 48, 64, 128, 256, 512};
// return false (launching nothing) for other sizes.
template <typename T>
bool fast_fft_available(int nx, int ny, int nz);
template <typename T>
bool fast_fft_y(const GridDesc<T>& g, int dir, int c, hipStream_t s);
template <typename T>
bool fast_fft_z_solve(const GridDesc<T>& g, SolveCoef sc, bool project, hipStream_t s);
template <typename T>
bool fast_fft_x_forward(const GridDesc<T>& g, const T* in, int c, hipStream_t s);
template <typename T>
bool fast_fft_x_inverse(const GridDesc<T>& g, T* out, bool accumulate, int c, hipStream_t s);

// ------------------------------------------------------------ grid kernels
template <typename T>
void launch_rhs(const GridDesc<T>& g, const RhsCoef& c, const RhsBlobs& rb, hipStream_t s);
template <typename T>
void launch_spread_overflow(const GridDesc<T>& g, const RhsBlobs& rb, hipStream_t s);
template <typename T>
void launch_equilibrium_noise(const GridDesc<T>& g, double sd, NoiseKey key, hipStream_t s);
template <typename T>
void launch_zero(T* p, long long n, hipStream_t s);
template <typename T>
void launch_axpy(T* y, const T* x, long long n, hipStream_t s);

// spread: field += h^-3 * prod(phi) * val, val_a = (F ? F[b][a] : 1) * (coef ? coef[b] : 1);
// deriv: the a-axis weight of component a is phi'(d)/h (thermal drift).
template <typename T>
void launch_spread(const GridDesc<T>& g, T* field, int kernel, int nb, const double* q,
                   const double* F, const double* coef, bool deriv, hipStream_t s);
// gather: out[b][a] = sum prod(phi) f_a (or of (L f)_a with laplacian = true)
template <typename T>
void launch_gather(const GridDesc<T>& g, const T* field, int kernel, int nb, const double* q,
                   double* out, bool laplacian, hipStream_t s);

// ------------------------------------------------------------ reductions
// acc[0..2] += rho h^3 sum v; acc[3] += rho h^3 sum v^2 / 2;
// acc[4] = max |v| (as bits), acc[5] = max |Dv| (as bits)
template <typename T>
void launch_field_diag(const GridDesc<T>& g, double rho, double* acc, hipStream_t s);

// ----------------------------------------------------------- blob kernels
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
    double *c5, *cdrift;                   // per-blob coefficients
    unsigned int* flag;                    // numeric error flag
    // spread inside the right-hand-side kernel
    double* stc;                           // max_nb * 3 * kStcPerComp
    int* chunk_count;                      // n_chunks + 1 (the last is the overflow count)
    int* chunk_list;                       // n_chunks * max_nb
    int* ovf_list;                         // 2 * ovf_cap
    int ovf_cap;
};

// Cell list of the pair forces: n[a] cells of width >= the cutoff per axis
// (at least 3), heads[cell] = (stamp << 32 | first blob), next[blob]. With
// heads == NULL the forces use the all-pairs kernel.
struct CellGrid {
    int n[3];
    double inv_size[3];
    unsigned long long* heads;
    int* next;
};
void launch_forces(const BlobParams& bp, const BlobBufs& b, const CellGrid& cg, unsigned int stamp, hipStream_t s);
void launch_inertial_dp(const BlobParams& bp, const BlobBufs& b, hipStream_t s);
void launch_inertial_dp2(const BlobParams& bp, const BlobBufs& b, hipStream_t s);
void launch_inertial_u(const BlobParams& bp, const BlobBufs& b, hipStream_t s);
void launch_blob_diag(int nb, const double* me, const double* u, double* acc, hipStream_t s);

// Fused gathers of the step (one 16-lane group per blob component):
// J^n v^n with the predictor; J^{n+1/2} v^n with the RHS stencils and z-chunk
// bins; J^{n+1/2} v^{n+1} with the position update (which also clears the
// first n_clear bin counters for the next step).
template <typename T>
void launch_gather_predict(const GridDesc<T>& g, int kernel, const BlobParams& bp, const BlobBufs& bb,
                           hipStream_t s);
template <typename T>
void launch_gather_bins(const GridDesc<T>& g, int kernel, const BlobParams& bp, const BlobBufs& bb, int cap,
                        hipStream_t s);
template <typename T>
void launch_gather_final(const GridDesc<T>& g, int kernel, const BlobParams& bp, const BlobBufs& bb, int n_clear,
                         hipStream_t s);
// z-chunk bins of the RHS spread (positions qh); counters must start at zero.
void launch_bins(int kernel, int nb, int nz, double h, const double* qh, int cap, int* chunk_count,
                 int* chunk_list, hipStream_t s);

}  // namespace icm
