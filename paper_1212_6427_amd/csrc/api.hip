// Context and C ABI of the ICM library (declared in include/icm.h).
//
// A context owns one HIP stream binding and a device workspace carved into
// per-replica field buffers (v, rhs, aux, spectrum), FFT twiddles, difference
// symbols and FP64 blob arrays. icm_step enqueues, for every replica, the
// nine steps of the Summary of Algorithm (Sec. III.C) as a fixed sequence of
// kernels; no host synchronisation happens inside a step.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/icm.h"
#include "icm_internal.h"

using icm::cplx;

namespace {

// message of the last failing call without a context: a fixed buffer, so
// that recording an error allocates nothing
thread_local char g_last_error[512] = "no error";

void set_last_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

struct Replica {
    icm_replica_params p;
    icm::CellGrid cells{};     // pair-force cell list (heads == NULL: all pairs)
    int max_nb = 0;
    int nb = 0;
    int64_t step = 0;
    int zc_tuned = 0;        // RHS z chunk from the autotuner (0: by batch size)
    bool any_me = false;
    double m_f = 0, mt_f = 0;
    icm::GridDesc<float> gf{};
    icm::GridDesc<double> gd{};
    icm::BlobBufs bb{};
    double* diag = nullptr;  // 16 doubles
    unsigned long long* d_step = nullptr;  // device step counter
    int slot = 0;            // index of the replica's descriptor in the device array
    bool tab_owner = false;  // builds the projection-kernel table of its grid shape
};

// Replicas stepped by the same launches: equal grid shape, kernel and
// advection setting. Their descriptors occupy slots [first, first + count)
// of the device array, the n_me replicas with a blob of nonzero excess mass
// first: the inertial correction (steps 4-8) is launched over those slots
// only, every other launch of the step over all of them.
struct BatchInfo {
    int n[3];
    int kernel;
    bool adv;
    int first, count;
    int max_nb;
    bool any_cells, any_all_pairs;
    int n_me;                // leading replicas on the inertial path
    int me_max_nb;           // their largest blob count
    bool table;              // their step 5 through the projection-kernel table
    std::vector<int> reps;   // inertial replicas first
};

}  // namespace

struct icm_ctx {
    // per-phase kernel timing (icm_set_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double phase_ms[16] = {0};
    int64_t phase_n[16] = {0};
    int32_t precision = ICM_FP64;
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool owns_ws = false;
    bool error_state = false;
    std::vector<Replica> reps;
    std::string err = "no error";
    // device descriptor array (RepDesc<float> or RepDesc<double> per slot)
    void* d_desc = nullptr;
    std::vector<unsigned char> h_desc;
    std::vector<BatchInfo> batches;
    // captured step (icm_step with ICM_STEP_GRAPH); batches after the first
    // are recorded on branch streams, so they are parallel branches of the
    // graph
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> branch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

icm_status fail(icm_ctx* c, icm_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        set_last_error(buf);
    return st;
}

#define HIP_TRY(ctx, call)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            if (ctx) (ctx)->error_state = true;                                                 \
            return fail(ctx, ICM_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
        }                                                                                       \
    } while (0)

// ------------------------------------------------------------ validation
using icm::factor_plan;

// Nodes per axis of a replica's stencil: the split three-point kernel
// (kernel_shift > 0) runs on the four-node layout.
int stencil_width(const icm_replica_params& p) { return p.kernel == 3 && p.kernel_shift > 0 ? 4 : p.kernel; }

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on the
// Legendre polynomial from the Chebyshev-like first guess
// cos(pi (i + 3/4) / (n + 1/2)), the recurrence
// (k + 1) P_{k+1} = (2k + 1) x P_k - k P_{k-1}, and w = 2 / ((1 - x^2) P_n'^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Sum over nodes of phi^2 averaged over the blob position in a cell (the
// constant of Eq. (JS_invariance) for the Peskin kernels). For the split
// kernel (Sec. III.A.2) the square of the mean of the two shifted copies
// averages to (1 + 2 A(sigma)) / 4, A(sigma) the integral of
// phi3(t) phi3(t + sigma) over t, integrated here by 24-point Gauss-Legendre
// on each interval between the kinks of the two factors (smooth inside).
double mean_sum_phi_sq(const icm_replica_params& p) {
    if (stencil_width(p) == p.kernel) return p.kernel == 3 ? 0.5 : 0.375;
    const double sg = p.kernel_shift;
    const double lo = std::max(-1.5, -1.5 - sg), hi = std::min(1.5, 1.5 - sg);
    std::vector<double> cut = {lo, hi};
    for (double b : {-0.5, 0.5, -0.5 - sg, 0.5 - sg})
        if (b > lo && b < hi) cut.push_back(b);
    std::sort(cut.begin(), cut.end());
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    double A = 0.0;
    for (size_t i = 0; i + 1 < cut.size(); ++i) {
        const double a = cut[i], b = cut[i + 1], m = 0.5 * (a + b), r = 0.5 * (b - a);
        if (r <= 0) continue;
        double s = 0.0;
        for (int k = 0; k < (int)gx.size(); ++k) {
            const double t = m + r * gx[k];
            s += gw[k] * icm::phi3(t) * icm::phi3(t + sg);
        }
        A += r * s;
    }
    return 0.25 * (1.0 + 2.0 * A);
}

icm_status validate(int32_t n_rep, const icm_replica_params* p, const int32_t* max_blobs, int32_t precision) {
    if (n_rep < 1) return fail(nullptr, ICM_E_INVALID, "n_rep must be >= 1 (got %d)", n_rep);
    if (!p || !max_blobs) return fail(nullptr, ICM_E_INVALID, "params and max_blobs must not be NULL");
    if (precision != ICM_FP64 && precision != ICM_FP32_GRID)
        return fail(nullptr, ICM_E_INVALID, "precision must be ICM_FP64 or ICM_FP32_GRID");
    for (int r = 0; r < n_rep; ++r) {
        const icm_replica_params& q = p[r];
        for (int a = 0; a < 3; ++a) {
            icm::FFTPlan pl;
            const int n = q.n[a];
            if (n < 4 || n > 512 || (n & 1) || !factor_plan(n, pl))
                return fail(nullptr, ICM_E_INVALID,
                            "replica %d: N[%d] = %d must be even, in [4, 512], with prime factors 2 and 3 only", r,
                            a, n);
        }
        if (q.kernel != 3 && q.kernel != 4) return fail(nullptr, ICM_E_INVALID, "replica %d: kernel must be 3 or 4", r);
        if (!(q.kernel_shift >= 0 && q.kernel_shift <= 1) || (q.kernel == 4 && q.kernel_shift != 0))
            return fail(nullptr, ICM_E_INVALID,
                        "replica %d: kernel_shift must be in [0, 1], and 0 with the four-point kernel", r);
        if (!(q.h > 0) || !(q.rho > 0) || !(q.eta >= 0) || !(q.kT >= 0) || !(q.dt > 0))
            return fail(nullptr, ICM_E_INVALID, "replica %d: need h > 0, rho > 0, eta >= 0, kT >= 0, dt > 0", r);
        if (q.slip < ICM_SLIP_NONE || q.slip > ICM_SLIP_FULL)
            return fail(nullptr, ICM_E_INVALID, "replica %d: slip must be ICM_SLIP_NONE/VISCOUS/FULL", r);
        if (q.thermal_drift != 0 && q.thermal_drift != 1)
            return fail(nullptr, ICM_E_INVALID, "replica %d: thermal_drift must be 0 or 1", r);
        if (q.advection > 1) return fail(nullptr, ICM_E_INVALID, "replica %d: advection must be 0 or 1", r);
        if (!(q.wca_eps >= 0)) return fail(nullptr, ICM_E_INVALID, "replica %d: wca_eps must be >= 0", r);
        if (q.wca_eps > 0) {
            const double rc = std::pow(2.0, 1.0 / 6.0) * q.wca_sigma;
            const double lmin = q.h * std::min(q.n[0], std::min(q.n[1], q.n[2]));
            if (!(q.wca_sigma > 0) || !(rc < 0.5 * lmin))
                return fail(nullptr, ICM_E_INVALID, "replica %d: need wca_sigma > 0 and cutoff < half the box", r);
        }
        if (max_blobs[r] < 0 || max_blobs[r] >= (1 << icm::kHeadBlobBits))
            return fail(nullptr, ICM_E_INVALID, "replica %d: max_blobs must be in [0, 2^%d)", r, icm::kHeadBlobBits);
    }
    return ICM_OK;
}

// ------------------------------------------------------- workspace carving
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename U>
    U* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        U* r = base ? reinterpret_cast<U*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(U);
        return r;
    }
};

template <typename T>
void carve_grid(Carver& cv, const icm_replica_params& p, icm::GridDesc<T>& g) {
    icm::grid_shape(g, p.n, p.h);
    g.hs = stencil_width(p) == p.kernel ? 0.0 : 0.5 * p.kernel_shift;
    g.v = cv.take<T>(3 * g.ncell);
    g.rhs = cv.take<T>(3 * g.ncell);
    g.aux = cv.take<T>(3 * g.ncell);
    g.spec = cv.take<cplx<T>>(3 * g.nspec);
    g.nyq = g.fast ? cv.take<cplx<T>>(3 * (long long)g.nz * g.ny) : nullptr;
    g.adv = p.advection ? cv.take<T>(3 * g.ncell) : nullptr;
    g.adv_hist = p.advection ? cv.take<unsigned int>(1) : nullptr;
    // FP32 grids carry the mean velocity (the k = 0 mode) in FP64
    g.k0 = sizeof(T) == 4 ? cv.take<double>(9) : nullptr;
    g.twx = cv.take<cplx<T>>(g.nx);
    g.twy = cv.take<cplx<T>>(g.ny);
    g.twz = cv.take<cplx<T>>(g.nz);
    g.dx_hat = cv.take<cplx<T>>(g.W);
    g.dy_hat = cv.take<cplx<T>>(g.ny);
    g.dz_hat = cv.take<cplx<T>>(g.nz);
    g.lx = cv.take<T>(g.W);
    g.ly = cv.take<T>(g.ny);
    g.lz = cv.take<T>(g.nz);
}

void carve_blobs(Carver& cv, int max_nb, const int n[3], icm::BlobBufs& b, double*& diag) {
    const size_t n3 = 3 * (size_t)max_nb;
    const int nbins = icm::rhs_bins(n[0], n[1], n[2]);
    b.stc = cv.take<double>((size_t)max_nb * 3 * icm::kStcPerComp);
    b.bin_count = cv.take<int>(nbins + 1);
    b.bin_list = cv.take<int>((size_t)nbins * icm::kRhsTileCap);
    // the stencils of a blob cover at most five nodes per axis, which meet
    // at most three tiles or chunks (two, unless a short last one lies
    // between them), so a blob is listed in (and can overflow) at most 27
    // bins
    b.ovf_cap = 27 * std::max(max_nb, 1);
    b.ovf_list = cv.take<int>(2 * (size_t)b.ovf_cap);
    b.q = cv.take<double>(n3);
    b.u = cv.take<double>(n3);
    b.fconst = cv.take<double>(n3);
    b.lag = cv.take<double>(n3);
    b.qh = cv.take<double>(n3);
    b.qw = cv.take<double>(n3);
    b.F = cv.take<double>(n3);
    b.Jn = cv.take<double>(n3);
    b.Jhvn = cv.take<double>(n3);
    b.Jhvt = cv.take<double>(n3);
    b.du = cv.take<double>(n3);
    b.dp = cv.take<double>(n3);
    b.dp2 = cv.take<double>(n3);
    b.g = cv.take<double>(n3);
    b.Jhvnew = cv.take<double>(n3);
    b.JLvt = cv.take<double>(n3);
    b.me = cv.take<double>(max_nb);
    b.c5 = cv.take<double>(max_nb);
    b.cdrift = cv.take<double>(max_nb);
    b.flag = cv.take<unsigned int>(1);
    diag = cv.take<double>(16);
}

// Cell list for the WCA pairs: cells at least one cutoff wide, at most 2^21
// of them, and at least 3 per axis (else the all-pairs kernel is used).
void carve_cells(Carver& cv, const icm_replica_params& p, int max_nb, icm::CellGrid& cg) {
    cg.heads = nullptr;
    cg.next = nullptr;
    if (!(p.wca_eps > 0) || max_nb < 2) return;
    const double rc = std::pow(2.0, 1.0 / 6.0) * p.wca_sigma;
    long long total = 1;
    for (int a = 0; a < 3; ++a) {
        const double L = p.n[a] * p.h;
        cg.n[a] = std::max(1, (int)std::floor(L / rc));
    }
    while ((long long)cg.n[0] * cg.n[1] * cg.n[2] > (1LL << 21)) {
        for (int a = 0; a < 3; ++a) cg.n[a] = std::max(1, cg.n[a] / 2);
    }
    if (cg.n[0] < 3 || cg.n[1] < 3 || cg.n[2] < 3) return;
    for (int a = 0; a < 3; ++a) {
        cg.inv_size[a] = cg.n[a] / (p.n[a] * p.h);
        total *= cg.n[a];
    }
    cg.heads = cv.take<unsigned long long>((size_t)total);
    cg.next = cv.take<int>((size_t)max_nb);
    if (!cv.base) cg.heads = reinterpret_cast<unsigned long long*>(1);  // sizing pass: mark as used
}

size_t desc_bytes(int32_t precision) {
    return precision == ICM_FP64 ? sizeof(icm::RepDesc<double>) : sizeof(icm::RepDesc<float>);
}

size_t layout(int32_t n_rep, const icm_replica_params* p, const int32_t* max_blobs, int32_t precision, void* base,
              std::vector<Replica>* reps, void** d_desc = nullptr) {
    Carver cv(base);
    void* desc = cv.take<unsigned char>(desc_bytes(precision) * (size_t)n_rep);
    if (d_desc) *d_desc = desc;
    unsigned long long* steps = cv.take<unsigned long long>((size_t)n_rep);
    if (reps)
        for (int r = 0; r < n_rep; ++r) (*reps)[r].d_step = steps + r;
    for (int r = 0; r < n_rep; ++r) {
        Replica tmp;
        Replica& R = reps ? (*reps)[r] : tmp;
        if (precision == ICM_FP64)
            carve_grid(cv, p[r], R.gd);
        else
            carve_grid(cv, p[r], R.gf);
        carve_blobs(cv, max_blobs[r], p[r].n, R.bb, R.diag);
        carve_cells(cv, p[r], max_blobs[r], R.cells);
    }
    // projection-kernel tables, one per grid shape that holds a replica of at
    // most kTabMaxBlobs blobs and at most kTabMaxCells cells
    const size_t word = precision == ICM_FP64 ? sizeof(double) : sizeof(float);
    std::vector<std::pair<std::array<int, 3>, void*>> shapes;
    for (int r = 0; r < n_rep; ++r) {
        const long long nc = (long long)p[r].n[0] * p[r].n[1] * p[r].n[2];
        if (max_blobs[r] > icm::kTabMaxBlobs || nc > icm::kTabMaxCells) continue;
        const std::array<int, 3> key = {p[r].n[0], p[r].n[1], p[r].n[2]};
        void* tab = nullptr;
        bool found = false;
        for (auto& s : shapes)
            if (s.first == key) {
                tab = s.second;
                found = true;
            }
        const bool owner = !found;
        if (owner) {
            tab = cv.take<unsigned char>(9 * (size_t)nc * word);
            shapes.push_back({key, tab});
        }
        if (reps) {
            Replica& R = (*reps)[r];
            R.tab_owner = owner;
            if (precision == ICM_FP64)
                R.gd.ptab = static_cast<const double*>(tab);
            else
                R.gf.ptab = static_cast<const float*>(tab);
        }
    }
    return (cv.off + 255) & ~size_t(255);
}

// ---------------------------------------------------------- host tables
template <typename T>
icm_status upload_tables(icm_ctx* c, const icm::GridDesc<T>& g) {
    const long double pi = 3.141592653589793238462643383279502884L;
    auto tw = [&](int n) {
        std::vector<cplx<T>> t(n);
        for (int m = 0; m < n; ++m) {
            const long double th = 2.0L * pi * (long double)m / (long double)n;
            t[m] = {(T)cosl(th), (T)(-sinl(th))};
        }
        return t;
    };
    // Dhat = (e^{i theta} - 1)/h = (-2 sin^2(theta/2) + i sin theta)/h,
    // lambda = 4 sin^2(theta/2) / h^2.
    auto sym = [&](int n, int count, std::vector<cplx<T>>& d, std::vector<T>& l) {
        d.resize(count);
        l.resize(count);
        for (int m = 0; m < count; ++m) {
            const long double th = 2.0L * pi * (long double)m / (long double)n;
            const long double s2 = sinl(0.5L * th);
            d[m] = {(T)(-2.0L * s2 * s2 / g.h), (T)(sinl(th) / g.h)};
            l[m] = (T)(4.0L * s2 * s2 / ((long double)g.h * g.h));
        }
    };
    const hipStream_t s = c->stream;
    auto tx = tw(g.nx), ty = tw(g.ny), tz = tw(g.nz);
    std::vector<cplx<T>> dx, dy, dz;
    std::vector<T> lx, ly, lz;
    sym(g.nx, g.W, dx, lx);
    sym(g.ny, g.ny, dy, ly);
    sym(g.nz, g.nz, dz, lz);
    HIP_TRY(c, hipMemcpyAsync((void*)g.twx, tx.data(), tx.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.twy, ty.data(), ty.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.twz, tz.data(), tz.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.dx_hat, dx.data(), dx.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.dy_hat, dy.data(), dy.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.dz_hat, dz.data(), dz.size() * sizeof(cplx<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.lx, lx.data(), lx.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.ly, ly.data(), ly.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync((void*)g.lz, lz.data(), lz.size() * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));  // host vectors go out of scope
    return ICM_OK;
}

icm::BlobParams blob_params(const Replica& R) {
    icm::BlobParams bp;
    bp.nb = R.nb;
    bp.dt = R.p.dt;
    bp.rho = R.p.rho;
    bp.eta = R.p.eta;
    bp.kT = R.p.kT;
    for (int a = 0; a < 3; ++a) {
        bp.box[a] = R.p.n[a] * R.p.h;
        bp.spring_c[a] = R.p.spring_center[a];
    }
    bp.wca_eps = R.p.wca_eps;
    bp.wca_sigma = R.p.wca_sigma;
    bp.spring_k = R.p.spring_k;
    bp.slip = R.p.slip;
    return bp;
}

icm::NoiseKey noise_key(const Replica& R, int64_t step) {
    icm::NoiseKey k;
    k.k0 = (uint32_t)(R.p.seed & 0xffffffffu);
    k.k1 = (uint32_t)(R.p.seed >> 32);
    k.step_lo = (uint32_t)((uint64_t)step & 0xffffffffu);
    k.step_hi = (uint32_t)((uint64_t)step >> 32);
    k.rep_tag = R.p.replica_id << 4;
    return k;
}

template <typename T>
icm::GridDesc<T>& grid_of(Replica& R);
template <>
icm::GridDesc<float>& grid_of<float>(Replica& R) { return R.gf; }
template <>
icm::GridDesc<double>& grid_of<double>(Replica& R) { return R.gd; }

hipEvent_t take_event(icm_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Run f (which enqueues kernels on s); with timing on, bracket it by events.
template <class F>
void timed(icm_ctx* c, int phase, hipStream_t s, F&& f) {
    if (!c || !c->timing) {
        f();
        return;
    }
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) {
        f();
        return;
    }
    (void)hipEventRecord(a, s);
    f();
    (void)hipEventRecord(b, s);
    c->pending.push_back({phase, {a, b}});
}

// Fold finished event pairs into the per-phase totals (stream synchronised).
void harvest_timing(icm_ctx* c) {
    for (auto& p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            c->phase_ms[p.first] += ms;
            c->phase_n[p.first] += 1;
        }
    }
    c->pending.clear();
    c->ev_used = 0;
}

// --------------------------------------------------------- descriptors
template <typename T>
icm::RepDesc<T> build_desc(const Replica& R) {
    icm::RepDesc<T> d{};
    d.g = grid_of<T>(const_cast<Replica&>(R));
    const icm::GridDesc<T>& g = d.g;
    const icm_replica_params& p = R.p;
    d.rc.rho_dt = p.rho / p.dt;
    d.rc.half_eta_h2 = 0.5 * p.eta / (p.h * p.h);
    d.rc.noise = p.kT > 0 ? std::sqrt(p.kT * p.eta / (p.h * p.h * p.h * p.dt)) / p.h : 0.0;
    d.rc.adv = p.advection ? p.rho / p.h : 0.0;
    for (int a = 0; a < 3; ++a) d.rc.body[a] = p.body_force[a];
    d.rc.key = noise_key(R, 0);
    const icm::BlobBufs& b = R.bb;
    const int nbins = icm::rhs_bins(g.nx, g.ny, g.nz);  // the overflow count follows the bins
    d.rb.nb = R.nb;
    d.rb.kernel = stencil_width(p);
    d.rb.stc = b.stc;
    d.rb.F = b.F;
    d.rb.cdrift = (p.kT > 0 && p.thermal_drift) ? b.cdrift : nullptr;
    d.rb.bin_count = b.bin_count;
    d.rb.bin_list = b.bin_list;
    d.rb.ovf_count = b.bin_count + nbins;
    d.rb.ovf_list = b.ovf_list;
    d.rb.ovf_cap = b.ovf_cap;
    d.bp = blob_params(R);
    d.bb = b;
    d.cg = R.cells;
    const double inv_n = 1.0 / (double)g.ncell;
    d.solve[icm::kSolveH1] = icm::SolveCoef{p.rho / p.dt, 0.5 * p.eta, inv_n};
    d.solve[icm::kSolveP] = icm::SolveCoef{1.0, 0.0, inv_n};
    d.solve[icm::kSolveH2] = icm::SolveCoef{p.rho, 0.5 * p.dt * p.eta, inv_n};
    const bool pairs = p.wca_eps > 0 && R.nb > 1;
    d.pair_mode = !pairs ? 0 : (R.cells.heads ? 1 : 2);
    d.step = R.d_step;
    return d;
}

// FP32-grid replicas carry their mean velocity in FP64; after the field
// was set from outside the step, re-derive it from the stored field.
icm_status reset_carry(icm_ctx* c, Replica& R, hipStream_t s) {
    if (c->precision == ICM_FP64) return ICM_OK;
    HIP_TRY(c, hipMemsetAsync(R.diag, 0, 16 * sizeof(double), s));
    icm::launch_carry_init(R.gf, R.p.rho, R.diag, s);
    HIP_TRY(c, hipGetLastError());
    return ICM_OK;
}

void drop_graph(icm_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// z chunk of the RHS kernel by batch size: the longest of 16, 8, 4 planes
// that still gives the launch at least 512 workgroups (two per compute
// unit); the 16-plane chunk amortises each chunk's prologue best.
int default_zc(const int n[3], int nrep) {
    const long long tiles = (long long)((n[0] + 31) / 32) * ((n[1] + 15) / 16) * (long long)nrep;
    int zc = icm::kRhsZChunk;
    while (zc > icm::kRhsZChunkMin && tiles * ((n[2] + zc - 1) / zc) < 512) zc /= 2;
    return zc;
}

// Group the replicas into batches and upload their descriptors (after any
// change of blob counts or masses). Drops a captured step.
template <typename T>
icm_status sync_batches_t(icm_ctx* c) {
    drop_graph(c);
    c->batches.clear();
    for (int r = 0; r < (int)c->reps.size(); ++r) {
        const Replica& R = c->reps[r];
        BatchInfo* hit = nullptr;
        for (BatchInfo& B : c->batches)
            if (B.n[0] == R.p.n[0] && B.n[1] == R.p.n[1] && B.n[2] == R.p.n[2] && B.kernel == stencil_width(R.p) &&
                B.adv == (R.p.advection != 0))
                hit = &B;
        if (!hit) {
            BatchInfo B{};
            for (int a = 0; a < 3; ++a) B.n[a] = R.p.n[a];
            B.kernel = stencil_width(R.p);
            B.adv = R.p.advection != 0;
            c->batches.push_back(B);
            hit = &c->batches.back();
        }
        hit->reps.push_back(r);
    }
    // inertial replicas first (a stable order within each part)
    for (BatchInfo& B : c->batches)
        std::stable_partition(B.reps.begin(), B.reps.end(), [c](int r) { return c->reps[r].any_me; });
    // z chunk of the RHS kernel per batch: the autotuner's, else by size
    for (BatchInfo& B : c->batches) {
        int zc = c->reps[B.reps[0]].zc_tuned;
        if (zc <= 0) zc = default_zc(B.n, (int)B.reps.size());
        for (int r : B.reps) grid_of<T>(c->reps[r]).zc = zc;
    }
    std::vector<icm::RepDesc<T>> h(c->reps.size());
    int slot = 0;
    for (BatchInfo& B : c->batches) {
        B.first = slot;
        B.count = (int)B.reps.size();
        B.max_nb = B.me_max_nb = B.n_me = 0;
        B.any_cells = B.any_all_pairs = false;
        B.table = true;
        for (int r : B.reps) {
            Replica& R = c->reps[r];
            R.slot = slot;
            h[slot] = build_desc<T>(R);
            B.max_nb = std::max(B.max_nb, R.nb);
            B.any_cells = B.any_cells || h[slot].pair_mode == 1;
            B.any_all_pairs = B.any_all_pairs || h[slot].pair_mode == 2;
            if (R.any_me) {
                ++B.n_me;
                B.me_max_nb = std::max(B.me_max_nb, R.nb);
                B.table = B.table && h[slot].g.ptab != nullptr;
            }
            ++slot;
        }
    }
    const size_t bytes = h.size() * sizeof(icm::RepDesc<T>);
    c->h_desc.resize(bytes);
    std::memcpy(c->h_desc.data(), h.data(), bytes);
    HIP_TRY(c, hipMemcpyAsync(c->d_desc, c->h_desc.data(), bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ICM_OK;
}

icm_status sync_batches(icm_ctx* c) {
    return c->precision == ICM_FP64 ? sync_batches_t<double>(c) : sync_batches_t<float>(c);
}

template <typename T>
icm::Batch<T> batch_view(icm_ctx* c, int first, int count, const Replica& R0, int max_nb, bool cells, bool all_pairs) {
    icm::Batch<T> B;
    B.d = static_cast<const icm::RepDesc<T>*>(c->d_desc) + first;
    B.nrep = count;
    B.g = grid_of<T>(const_cast<Replica&>(R0));
    B.kernel = stencil_width(R0.p);
    B.max_nb = max_nb;
    B.any_cells = cells;
    B.any_all_pairs = all_pairs;
    B.one = count == 1 ? reinterpret_cast<const icm::RepDesc<T>*>(c->h_desc.data()) + first : nullptr;
    return B;
}

template <typename T>
icm::Batch<T> batch_of(icm_ctx* c, const BatchInfo& bi) {
    return batch_view<T>(c, bi.first, bi.count, c->reps[bi.reps[0]], bi.max_nb, bi.any_cells, bi.any_all_pairs);
}

// The one-replica batch of replica R (set-up work outside the step).
template <typename T>
icm::Batch<T> single(icm_ctx* c, const Replica& R) {
    return batch_view<T>(c, R.slot, 1, R, R.nb, false, false);
}

// Forward transform, spectral solve, inverse transform.
template <typename T>
void enqueue_fft_solve(icm_ctx* c, const icm::Batch<T>& B, int in, int out, int accumulate, int solve,
                       hipStream_t s) {
    timed(c, ICM_PHASE_FFT_X_FWD, s, [&] { icm::launch_fft_x_forward(B, in, s); });
    timed(c, ICM_PHASE_FFT_Y_FWD, s, [&] { icm::launch_fft_y(B, -1, s); });
    timed(c, ICM_PHASE_FFT_Z_SOLVE, s,
          [&] { icm::launch_fft_z_solve(B, solve, true, s, solve == icm::kSolveH1 || solve == icm::kSolveH2); });
    timed(c, ICM_PHASE_FFT_Y_INV, s, [&] { icm::launch_fft_y(B, 1, s); });
    timed(c, ICM_PHASE_FFT_X_INV, s, [&] { icm::launch_fft_x_inverse(B, out, accumulate, s); });
}

// One step of Sec. III.C for every replica of a batch, enqueued on stream s.
// Nothing here reads host state that changes from step to step.
template <typename T>
void enqueue_step(icm_ctx* c, const BatchInfo& bi, hipStream_t s) {
    const icm::Batch<T> B = batch_of<T>(c, bi);
    using namespace icm;
    // Step 1: midpoint predictor with the one-body forces; J^{n+1/2} v^n (for
    // step 9) with the spread stencils and the cell lists; pair forces and
    // the RHS bins of the spread.
    timed(c, ICM_PHASE_GATHER, s, [&] { launch_gather_step1(B, s); });
    timed(c, ICM_PHASE_FORCES, s, [&] { launch_forces(B, s); });
    // Step 2: unperturbed fluid solve; S F and the thermal drift are spread
    // inside the right-hand-side kernel.
    timed(c, ICM_PHASE_RHS, s, [&] { launch_rhs(B, s); });
    timed(c, ICM_PHASE_SPREAD, s, [&] { launch_spread_overflow(B, s); });
    if (bi.adv) timed(c, ICM_PHASE_ADVECTION, s, [&] { launch_advect(B, s); });
    // Replicas with excess mass and at most kTabMaxBlobs blobs on a
    // register-resident grid keep the first solve in the spectrum: step 4
    // reads J v~ (and J L v~) from it, step 6's solve adds its own result to
    // it, and one inverse y and x pass then gives v^{n+1}.
    const bool spectral = bi.n_me > 0 && bi.table && bi.me_max_nb <= kTabMaxBlobs && B.g.fast;
    if (!spectral) {
        enqueue_fft_solve(c, B, kFieldRhs, kFieldV, 0, kSolveH1, s);
    } else {
        timed(c, ICM_PHASE_FFT_X_FWD, s, [&] { launch_fft_x_forward(B, kFieldRhs, s); });
        timed(c, ICM_PHASE_FFT_Y_FWD, s, [&] { launch_fft_y(B, -1, s); });
        timed(c, ICM_PHASE_FFT_Z_SOLVE, s, [&] { launch_fft_z_solve(B, kSolveH1, true, s, true); });
    }
    if (bi.n_me > 0) {
        // steps 4-8 over the leading replicas with excess mass only
        const icm::Batch<T> B = batch_view<T>(c, bi.first, bi.n_me, c->reps[bi.reps[0]], bi.me_max_nb, false, false);
        // Step 4: J^{n+1/2} v~, the slip correction and the excess momentum.
        if (spectral)
            timed(c, ICM_PHASE_GATHER, s, [&] { launch_spectral_gather(B, s); });
        else
            timed(c, ICM_PHASE_GATHER, s, [&] { launch_gather(B, kFieldV, kBlobQh, kBlobJhvt, false, s, kEpiDp); });
        // Step 5: dv~ = m~_f/(rho m~) P S dp, needed only as g = J dv~: for
        // few blobs through the projection-kernel table, else as a field;
        // with g, the step-6 source dp - m_e J dv~ and u^{n+1} (step 8).
        if (bi.table && bi.me_max_nb <= kTabMaxBlobs) {
            timed(c, ICM_PHASE_BLOB, s, [&] { launch_jps_table(B, s); });
        } else {
            timed(c, ICM_PHASE_FIELD_OPS, s, [&] { launch_zero(B, kFieldRhs, s); });
            timed(c, ICM_PHASE_SPREAD, s, [&] { launch_spread(B, kFieldRhs, kBlobQh, kBlobDp, kBlobC5, s); });
            enqueue_fft_solve(c, B, kFieldRhs, kFieldAux, 0, kSolveP, s);
            timed(c, ICM_PHASE_GATHER, s, [&] { launch_gather(B, kFieldAux, kBlobQh, kBlobG, false, s, kEpiDp2); });
            timed(c, ICM_PHASE_BLOB, s, [&] { launch_dp2_sum(B, s); });
        }
        // Step 6: (rho - dt/2 eta L) dv + dt G dpi = S (dp - m_e J dv~);
        // step 7: v^{n+1} = v~ + dv.
        if (spectral) {
            // the z pass forms the transform of the spread source from the
            // stencil records and adds its solve to the first one
            timed(c, ICM_PHASE_FFT_Z_SOLVE, s, [&] { (void)fast_fft_z_solve_from_blobs(B, kSolveH2, s, true, true); });
        } else {
            // dv written to aux by the last pass (for the lagged term of
            // step 9) and added to v
            timed(c, ICM_PHASE_FIELD_OPS, s, [&] { launch_zero(B, kFieldRhs, s); });
            timed(c, ICM_PHASE_SPREAD, s, [&] { launch_spread(B, kFieldRhs, kBlobQh, kBlobDp2, kBlobNone, s); });
            enqueue_fft_solve(c, B, kFieldRhs, kFieldAux, kXinvAlsoV, kSolveH2, s);
        }
    }
    if (spectral) {
        // one y and x inverse pass for the whole batch: v^{n+1} of the
        // replicas without excess mass from the first solve's spectrum
        // (untouched since), of the others from the sum of both solves
        timed(c, ICM_PHASE_FFT_Y_INV, s, [&] { launch_fft_y(B, 1, s); });
        timed(c, ICM_PHASE_FFT_X_INV, s, [&] { launch_fft_x_inverse(B, kFieldV, 0, s); });
    }
    // Step 9 (also the lagged term of the inertial replicas and the device
    // step counters).
    timed(c, ICM_PHASE_GATHER, s, [&] { launch_gather_final(B, bi.n_me, spectral, s); });
}

template <typename T>
void enqueue_all(icm_ctx* c, hipStream_t s) {
    for (const BatchInfo& bi : c->batches) enqueue_step<T>(c, bi, s);
}

// v (+)= P(field in) for one replica.
template <typename T>
void enqueue_project(icm_ctx* c, const Replica& R, int in, bool accumulate, hipStream_t s) {
    const icm::Batch<T> B = single<T>(c, R);
    icm::launch_fft_x_forward(B, in, s);
    icm::launch_fft_y(B, -1, s);
    icm::launch_fft_z_solve(B, icm::kSolveP, true, s);
    icm::launch_fft_y(B, 1, s);
    icm::launch_fft_x_inverse(B, icm::kFieldV, accumulate, s);
}

// v += P S (impulse) / rho with the impulse already in dp (ICM_BLOBS_KICK).
template <typename T>
void kick(icm_ctx* c, const Replica& R, hipStream_t s) {
    const icm::Batch<T> B = single<T>(c, R);
    icm::launch_zero(B, icm::kFieldRhs, s);
    icm::launch_spread(B, icm::kFieldRhs, icm::kBlobQ, icm::kBlobDp, icm::kBlobNone, s);
    enqueue_project<T>(c, R, icm::kFieldRhs, true, s);
}

// The projection-kernel tables: for each grid shape that has one, its first
// replica projects the unit impulse on face 0 of each component b with its
// own scratch fields (the fluid is at rest right after create), and the
// result, (P e_b)_a for a = x, y, z, is copied into the table.
template <typename T>
icm_status build_tables_t(icm_ctx* c) {
    hipStream_t s = c->stream;
    for (Replica& R : c->reps) {
        if (!R.tab_owner) continue;
        icm::GridDesc<T>& g = grid_of<T>(R);
        const size_t fb = 3 * (size_t)g.ncell * sizeof(T);
        const T one = 1;
        for (int b = 0; b < 3; ++b) {
            HIP_TRY(c, hipMemsetAsync(g.rhs, 0, fb, s));
            HIP_TRY(c, hipMemcpyAsync(g.rhs + (size_t)b * g.ncell, &one, sizeof(T), hipMemcpyHostToDevice, s));
            enqueue_project<T>(c, R, icm::kFieldRhs, false, s);
            HIP_TRY(c, hipGetLastError());
            HIP_TRY(c, hipMemcpyAsync(const_cast<T*>(g.ptab) + (size_t)b * 3 * g.ncell, g.v, fb,
                                      hipMemcpyDeviceToDevice, s));
            HIP_TRY(c, hipStreamSynchronize(s));  // `one` lives on the stack
        }
        HIP_TRY(c, hipMemsetAsync(g.v, 0, fb, s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return ICM_OK;
}

icm_status build_tables(icm_ctx* c) {
    return c->precision == ICM_FP64 ? build_tables_t<double>(c) : build_tables_t<float>(c);
}

// Record one step of every batch into a graph (kernel launches only; the
// step counters and all per-replica data live in device memory). Batches
// (one per grid shape, kernel and advection setting) touch disjoint memory,
// so each is its own branch of the graph: the first
// on the capture stream, the others on branch streams forked from it by an
// event and joined back at the end.
icm_status capture_step(icm_ctx* c) {
    drop_graph(c);
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const size_t nb = c->batches.size();
    while (c->branch.size() + 1 < nb) {
        hipStream_t st = nullptr;
        HIP_TRY(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->branch.push_back(st);
    }
    std::vector<hipEvent_t> ev(nb, nullptr);  // ev[0]: fork; ev[b]: end of branch b
    for (hipEvent_t& e : ev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
            return fail(c, ICM_E_DEVICE, "event creation failed");
        }
    }
    const hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
        c->error_state = true;
        return fail(c, ICM_E_DEVICE, "step capture failed: %s", hipGetErrorString(eb));
    }
    hipError_t err = hipSuccess;
    if (nb > 1) err = hipEventRecord(ev[0], c->cap_stream);
    for (size_t b = 1; b < nb && err == hipSuccess; ++b) err = hipStreamWaitEvent(c->branch[b - 1], ev[0], 0);
    for (size_t b = 0; b < nb && err == hipSuccess; ++b) {
        const hipStream_t s = b == 0 ? c->cap_stream : c->branch[b - 1];
        if (c->precision == ICM_FP64)
            enqueue_step<double>(c, c->batches[b], s);
        else
            enqueue_step<float>(c, c->batches[b], s);
        err = hipGetLastError();
    }
    for (size_t b = 1; b < nb && err == hipSuccess; ++b) {
        err = hipEventRecord(ev[b], c->branch[b - 1]);
        if (err == hipSuccess) err = hipStreamWaitEvent(c->cap_stream, ev[b], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    if (err != hipSuccess || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        c->error_state = true;
        return fail(c, ICM_E_DEVICE, "step capture failed: %s", hipGetErrorString(err != hipSuccess ? err : e));
    }
    c->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    return ICM_OK;
}

// ----------------------------------------------------------- autotuner
// Average time of one solve's five FFT passes (x, y, z with the projection,
// y inverse, x inverse) for the batch B with its current launch shapes, on
// the context's scratch fields. The x forward pass reads the right-hand-side
// field each time, so repeated unnormalised transforms stay finite.
template <typename T>
float time_fft(icm_ctx* c, const icm::Batch<T>& B, hipEvent_t ea, hipEvent_t eb) {
    using namespace icm;
    hipStream_t s = c->stream;
    auto once = [&] {
        launch_fft_x_forward(B, kFieldRhs, s);
        launch_fft_y(B, -1, s);
        launch_fft_z_solve(B, kSolveP, true, s);
        launch_fft_y(B, 1, s);
        launch_fft_x_inverse(B, kFieldAux, false, s);
    };
    constexpr int kReps = 10;
    once();  // warm-up
    (void)hipEventRecord(ea, s);
    for (int r = 0; r < kReps; ++r) once();
    (void)hipEventRecord(eb, s);
    if (hipEventSynchronize(eb) != hipSuccess) return -1.f;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) return -1.f;
    return ms * 1000.f / kReps;
}

// Average time of one right-hand-side launch of batch b with z chunk zc,
// each followed by one solve's five FFT passes as in the step (the RHS kernel
// timed alone finds different data in the caches, and such timings picked
// chunks that were slower in the step): the chunk is installed, the
// spread's bins computed for it (from stencil records at the current
// positions, which a step has not necessarily written yet, and the last
// step's forces) and cleared again afterwards.
template <typename T>
float time_rhs(icm_ctx* c, size_t b, int zc, hipEvent_t ea, hipEvent_t eb) {
    for (int r : c->batches[b].reps) c->reps[r].zc_tuned = zc;
    if (sync_batches(c) != ICM_OK) return -1.f;
    const BatchInfo& bi = c->batches[b];  // same grouping: the replicas did not change
    const icm::Batch<T> B = batch_of<T>(c, bi);
    hipStream_t s = c->stream;
    auto clear = [&] {
        for (int r : bi.reps) {
            const Replica& R = c->reps[r];
            (void)hipMemsetAsync(R.bb.bin_count, 0,
                                 (size_t)(icm::rhs_bins(R.p.n[0], R.p.n[1], R.p.n[2]) + 1) * sizeof(int), s);
        }
    };
    clear();
    icm::launch_stencil_records(B, s);
    icm::launch_bins(B, s);
    auto once = [&] {
        icm::launch_rhs(B, s);
        icm::launch_fft_x_forward(B, icm::kFieldRhs, s);
        icm::launch_fft_y(B, -1, s);
        icm::launch_fft_z_solve(B, icm::kSolveP, true, s);
        icm::launch_fft_y(B, 1, s);
        icm::launch_fft_x_inverse(B, icm::kFieldAux, 0, s);
    };
    once();  // warm-up
    constexpr int kReps = 10;
    (void)hipEventRecord(ea, s);
    for (int r = 0; r < kReps; ++r) once();
    (void)hipEventRecord(eb, s);
    clear();
    if (hipEventSynchronize(eb) != hipSuccess) return -1.f;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) return -1.f;
    return ms * 1000.f / kReps;
}

template <typename T>
icm_status autotune_t(icm_ctx* c, icm_tune_result* res, int32_t cap, int32_t* nres) {
    hipEvent_t ea = nullptr, eb = nullptr;
    HIP_TRY(c, hipEventCreate(&ea));
    if (hipEventCreate(&eb) != hipSuccess) {
        (void)hipEventDestroy(ea);
        return fail(c, ICM_E_DEVICE, "hipEventCreate failed");
    }
    std::vector<std::array<int, 3>> done;
    int count = 0;
    icm_status st = ICM_OK;
    for (const BatchInfo& bi : c->batches) {
        const std::array<int, 3> shape = {bi.n[0], bi.n[1], bi.n[2]};
        if (std::find(done.begin(), done.end(), shape) != done.end()) continue;
        done.push_back(shape);
        // all replicas of this shape, whichever batch holds them
        icm::Batch<T> B = batch_of<T>(c, bi);
        icm_tune_result r{};
        for (int a = 0; a < 3; ++a) r.n[a] = shape[a];
        const float t0 = time_fft<T>(c, B, ea, eb);
        if (t0 < 0) {
            st = fail(c, ICM_E_DEVICE, "autotune timing failed");
            break;
        }
        r.us_default = t0;
        icm::GridDesc<T>& g = B.g;
        if (g.fast) {
            r.tuned = 1;
            // z pass: plan size x columns; then y columns; then x threads.
            // Every candidate is timed over the whole five-pass round trip
            // (a pass timed alone keeps its working set in the last-level
            // cache, which the step does not), and replaces the current
            // choice only if it is at least 1% faster.
            const int zplans[2] = {1, 0};
            const int cols[3] = {8, 16, 32};
            const int xts[3] = {128, 256, 512};
            auto better = [](float t, float best) { return t >= 0 && t < 0.99f * best; };
            float best = t0;
            int bz = g.Bz, zs = g.zsmall;
            for (int zp : zplans)
                for (int cz : cols) {
                    if (zp == zs && cz == bz) continue;
                    g.zsmall = zp;
                    g.Bz = cz;
                    const float t = time_fft<T>(c, B, ea, eb);
                    if (better(t, best)) { best = t; bz = cz; zs = zp; }
                    g.zsmall = zs;
                    g.Bz = bz;
                }
            int by = g.By;
            for (int cy : cols) {
                if (cy == by) continue;
                g.By = cy;
                const float t = time_fft<T>(c, B, ea, eb);
                if (better(t, best)) { best = t; by = cy; }
                g.By = by;
            }
            int xt = g.xt;
            for (int x : xts) {
                if (x == xt) continue;
                g.xt = x;
                const float t = time_fft<T>(c, B, ea, eb);
                if (better(t, best)) { best = t; xt = x; }
                g.xt = xt;
            }
            g.xt = xt;
            r.us_tuned = time_fft<T>(c, B, ea, eb);
            for (Replica& R : c->reps)
                if (R.p.n[0] == shape[0] && R.p.n[1] == shape[1] && R.p.n[2] == shape[2]) {
                    icm::GridDesc<T>& gr = grid_of<T>(R);
                    gr.By = g.By;
                    gr.Bz = g.Bz;
                    gr.xt = g.xt;
                    gr.zsmall = g.zsmall;
                }
        } else {
            r.us_tuned = r.us_default;
        }
        r.y_columns = g.By;
        r.z_columns = g.Bz;
        r.z_small_plan = g.zsmall;
        r.x_threads = g.xt;
        if (res && count < cap) res[count] = r;
        ++count;
    }
    // RHS z chunk per batch: 16, 8 and 4 planes, each timed with its own
    // bins (RHS plus a solve's passes); the size-based choice stays unless
    // another makes that unit at least 1% faster
    for (size_t b = 0; b < c->batches.size() && st == ICM_OK; ++b) {
        const std::vector<int> reps = c->batches[b].reps;
        int n3[3];
        for (int a = 0; a < 3; ++a) n3[a] = c->batches[b].n[a];
        const int zdef = default_zc(n3, (int)reps.size());
        const float t0 = time_rhs<T>(c, b, zdef, ea, eb);
        if (t0 < 0) {
            st = fail(c, ICM_E_DEVICE, "autotune timing failed");
            break;
        }
        float best = t0;
        int bz = zdef;
        for (int zc : {16, 8, 4}) {
            if (zc == zdef) continue;
            const float t = time_rhs<T>(c, b, zc, ea, eb);
            if (t >= 0 && t < 0.99f * best) {
                best = t;
                bz = zc;
            }
        }
        for (int r : reps) c->reps[r].zc_tuned = bz;
        for (int e = 0; res && e < std::min(count, (int)cap); ++e)
            if (res[e].n[0] == n3[0] && res[e].n[1] == n3[1] && res[e].n[2] == n3[2] && res[e].rhs_z_chunk == 0) {
                res[e].rhs_z_chunk = bz;
                res[e].us_rhs_default = t0;
                res[e].us_rhs_tuned = best;
                break;
            }
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (st != ICM_OK) return st;
    if (nres) *nres = count;
    return sync_batches(c);
}

icm_status check_replica(icm_ctx* c, int32_t replica) {
    if (!c) return fail(nullptr, ICM_E_INVALID, "NULL context");
    if (replica < 0 || replica >= (int32_t)c->reps.size())
        return fail(c, ICM_E_INVALID, "replica %d out of range [0, %d)", replica, (int)c->reps.size());
    return ICM_OK;
}

size_t field_bytes(const icm_ctx* c, const Replica& R) {
    const long long ncell = (long long)R.p.n[0] * R.p.n[1] * R.p.n[2];
    return 3 * (size_t)ncell * (c->precision == ICM_FP64 ? sizeof(double) : sizeof(float));
}

void* field_ptr(icm_ctx* c, Replica& R) {
    return c->precision == ICM_FP64 ? (void*)R.gd.v : (void*)R.gf.v;
}
void* rhs_ptr(icm_ctx* c, Replica& R) {
    return c->precision == ICM_FP64 ? (void*)R.gd.rhs : (void*)R.gf.rhs;
}
unsigned int* adv_hist_of(const icm_ctx* c, const Replica& R) {
    return c->precision == ICM_FP64 ? R.gd.adv_hist : R.gf.adv_hist;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

icm_status icm_workspace_bytes(int32_t n_rep, const icm_replica_params* p, const int32_t* max_blobs,
                               int32_t precision, size_t* bytes) {
    icm_status st = validate(n_rep, p, max_blobs, precision);
    if (st != ICM_OK) return st;
    if (!bytes) return fail(nullptr, ICM_E_INVALID, "bytes must not be NULL");
    *bytes = layout(n_rep, p, max_blobs, precision, nullptr, nullptr);
    return ICM_OK;
}

icm_status icm_create(int32_t n_rep, const icm_replica_params* p, const int32_t* max_blobs, int32_t precision,
                      void* workspace, size_t bytes, void* stream, icm_ctx** out) {
    if (!out) return fail(nullptr, ICM_E_INVALID, "out must not be NULL");
    *out = nullptr;
    icm_status st = validate(n_rep, p, max_blobs, precision);
    if (st != ICM_OK) return st;
    const size_t need = layout(n_rep, p, max_blobs, precision, nullptr, nullptr);
    icm_ctx* c = new icm_ctx();
    c->precision = precision;
    c->stream = static_cast<hipStream_t>(stream);
    if (workspace) {
        if (bytes < need) {
            delete c;
            return fail(nullptr, ICM_E_NOMEM, "workspace of %zu bytes is smaller than the %zu required", bytes, need);
        }
        if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
            delete c;
            return fail(nullptr, ICM_E_INVALID, "workspace must be 256-byte aligned");
        }
        c->ws = workspace;
        c->ws_bytes = bytes;
    } else {
        hipError_t e = hipMalloc(&c->ws, need);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, ICM_E_NOMEM, "hipMalloc of %zu bytes failed: %s", need, hipGetErrorString(e));
        }
        c->owns_ws = true;
        c->ws_bytes = need;
    }
    c->reps.resize(n_rep);
    layout(n_rep, p, max_blobs, precision, c->ws, &c->reps, &c->d_desc);
    for (int r = 0; r < n_rep; ++r) {
        Replica& R = c->reps[r];
        R.p = p[r];
        R.max_nb = max_blobs[r];
        R.nb = 0;
        R.step = 0;
        R.m_f = p[r].rho * std::pow(p[r].h, 3) / std::pow(mean_sum_phi_sq(p[r]), 3);
        R.mt_f = 1.5 * R.m_f;
        st = (precision == ICM_FP64) ? upload_tables(c, R.gd) : upload_tables(c, R.gf);
        if (st != ICM_OK) {
            set_last_error(c->err.c_str());
            icm_destroy(c);
            return st;
        }
        const size_t fb = field_bytes(c, R);
        hipError_t e = hipMemsetAsync(field_ptr(c, R), 0, fb, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(R.bb.flag, 0, sizeof(unsigned int), c->stream);
        if (e == hipSuccess && R.cells.heads)
            e = hipMemsetAsync(R.cells.heads, 0,
                               sizeof(unsigned long long) * (size_t)R.cells.n[0] * R.cells.n[1] * R.cells.n[2],
                               c->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(R.bb.bin_count, 0,
                               sizeof(int) * (icm::rhs_bins(p[r].n[0], p[r].n[1], p[r].n[2]) + 1), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(R.d_step, 0, sizeof(unsigned long long), c->stream);
        if (e == hipSuccess && R.gf.k0 && precision == ICM_FP32_GRID)
            e = hipMemsetAsync(R.gf.k0, 0, 9 * sizeof(double), c->stream);
        if (e == hipSuccess && adv_hist_of(c, R))
            e = hipMemsetAsync(adv_hist_of(c, R), 0, sizeof(unsigned int), c->stream);
        if (e != hipSuccess) {
            snprintf(g_last_error, sizeof(g_last_error), "hipMemsetAsync failed: %s", hipGetErrorString(e));
            icm_destroy(c);
            return ICM_E_DEVICE;
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        set_last_error("stream synchronisation failed after create");
        icm_destroy(c);
        return ICM_E_DEVICE;
    }
    st = sync_batches(c);
    if (st == ICM_OK) st = build_tables(c);
    if (st != ICM_OK) {
        set_last_error(c->err.c_str());
        icm_destroy(c);
        return st;
    }
    *out = c;
    return ICM_OK;
}

icm_status icm_set_blobs(icm_ctx* c, int32_t replica, int32_t n_blobs, const double* q, const double* u,
                         const double* m_e, const double* f_const, uint32_t flags) {
    icm_status st = check_replica(c, replica);
    if (st != ICM_OK) return st;
    Replica& R = c->reps[replica];
    if (n_blobs < 0 || n_blobs > R.max_nb)
        return fail(c, ICM_E_INVALID, "n_blobs = %d outside [0, max_blobs = %d]", n_blobs, R.max_nb);
    if (n_blobs > 0 && !q) return fail(c, ICM_E_INVALID, "q must not be NULL");
    const bool dev = (flags & ICM_PTRS_DEVICE) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const size_t n3 = 3 * (size_t)n_blobs;
    hipStream_t s = c->stream;
    // masses are needed on the host for validation and coefficients
    std::vector<double> me(n_blobs, 0.0);
    if (m_e && n_blobs) {
        if (dev) {
            HIP_TRY(c, hipMemcpyAsync(me.data(), m_e, n_blobs * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(c, hipStreamSynchronize(s));
        } else {
            std::memcpy(me.data(), m_e, n_blobs * sizeof(double));
        }
    }
    for (int i = 0; i < n_blobs; ++i)
        if (!(me[i] > -R.m_f) || !std::isfinite(me[i]))
            return fail(c, ICM_E_INVALID, "blob %d: m_e = %g must exceed -m_f = %g", i, me[i], -R.m_f);
    std::vector<double> c5(n_blobs), cd(n_blobs);
    bool any = false;
    for (int i = 0; i < n_blobs; ++i) {
        c5[i] = R.mt_f / (R.p.rho * (me[i] + R.mt_f));
        cd[i] = R.p.kT * R.mt_f / (me[i] + R.mt_f);
        any = any || me[i] != 0.0;
    }
    if (n_blobs) {
        HIP_TRY(c, hipMemcpyAsync(R.bb.q, q, n3 * sizeof(double), kind, s));
        if (u)
            HIP_TRY(c, hipMemcpyAsync(R.bb.u, u, n3 * sizeof(double), kind, s));
        else
            HIP_TRY(c, hipMemsetAsync(R.bb.u, 0, n3 * sizeof(double), s));
        if (f_const)
            HIP_TRY(c, hipMemcpyAsync(R.bb.fconst, f_const, n3 * sizeof(double), kind, s));
        else
            HIP_TRY(c, hipMemsetAsync(R.bb.fconst, 0, n3 * sizeof(double), s));
        HIP_TRY(c, hipMemcpyAsync(R.bb.me, me.data(), n_blobs * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(R.bb.c5, c5.data(), n_blobs * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(R.bb.cdrift, cd.data(), n_blobs * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemsetAsync(R.bb.lag, 0, n3 * sizeof(double), s));
    }
    R.nb = n_blobs;
    R.any_me = any;
    if (c->precision == ICM_FP32_GRID)  // force sums of the carried mean (recomputed every step with blobs)
        HIP_TRY(c, hipMemsetAsync(R.gf.k0 + 3, 0, 6 * sizeof(double), s));
    st = sync_batches(c);
    if (st != ICM_OK) return st;
    if ((flags & ICM_BLOBS_KICK) && n_blobs) {
        // v += P S (m~_f u0) / rho
        std::vector<double> imp(n3, 0.0);
        if (u) {
            if (dev) {
                HIP_TRY(c, hipMemcpyAsync(imp.data(), u, n3 * sizeof(double), hipMemcpyDeviceToHost, s));
                HIP_TRY(c, hipStreamSynchronize(s));
            } else {
                std::memcpy(imp.data(), u, n3 * sizeof(double));
            }
        }
        for (auto& x : imp) x *= R.mt_f / R.p.rho;
        HIP_TRY(c, hipMemcpyAsync(R.bb.dp, imp.data(), n3 * sizeof(double), hipMemcpyHostToDevice, s));
        if (c->precision == ICM_FP64)
            kick<double>(c, R, s);
        else
            kick<float>(c, R, s);
        HIP_TRY(c, hipGetLastError());
        if (adv_hist_of(c, R)) HIP_TRY(c, hipMemsetAsync(adv_hist_of(c, R), 0, sizeof(unsigned int), s));
        st = reset_carry(c, R, s);
        if (st != ICM_OK) return st;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return ICM_OK;
}

icm_status icm_set_state(icm_ctx* c, int32_t replica, const void* v, const double* q, const double* u,
                         const double* lag_c, int64_t step, uint32_t flags) {
    icm_status st = check_replica(c, replica);
    if (st != ICM_OK) return st;
    Replica& R = c->reps[replica];
    const bool dev = (flags & ICM_PTRS_DEVICE) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const size_t n3 = 3 * (size_t)R.nb;
    hipStream_t s = c->stream;
    const size_t fb = field_bytes(c, R);
    if (flags & ICM_STATE_EQUILIBRIUM) {
        const double sd = std::sqrt(R.p.kT / (R.p.rho * R.p.h * R.p.h * R.p.h));
        if (c->precision == ICM_FP64) {
            icm::launch_equilibrium_noise(single<double>(c, R), sd, s);
            enqueue_project<double>(c, R, icm::kFieldRhs, false, s);
        } else {
            icm::launch_equilibrium_noise(single<float>(c, R), sd, s);
            enqueue_project<float>(c, R, icm::kFieldRhs, false, s);
        }
        HIP_TRY(c, hipGetLastError());
    } else if (v) {
        if (flags & ICM_STATE_PROJECT) {
            HIP_TRY(c, hipMemcpyAsync(rhs_ptr(c, R), v, fb, kind, s));
            if (c->precision == ICM_FP64)
                enqueue_project<double>(c, R, icm::kFieldRhs, false, s);
            else
                enqueue_project<float>(c, R, icm::kFieldRhs, false, s);
            HIP_TRY(c, hipGetLastError());
        } else {
            HIP_TRY(c, hipMemcpyAsync(field_ptr(c, R), v, fb, kind, s));
        }
    }
    // a new field starts the advective history again (first step: Euler)
    if (((flags & ICM_STATE_EQUILIBRIUM) || v) && adv_hist_of(c, R))
        HIP_TRY(c, hipMemsetAsync(adv_hist_of(c, R), 0, sizeof(unsigned int), s));
    if ((flags & ICM_STATE_EQUILIBRIUM) || v) {
        st = reset_carry(c, R, s);
        if (st != ICM_OK) return st;
    }
    if (q && n3) HIP_TRY(c, hipMemcpyAsync(R.bb.q, q, n3 * sizeof(double), kind, s));
    if (u && n3) HIP_TRY(c, hipMemcpyAsync(R.bb.u, u, n3 * sizeof(double), kind, s));
    if (lag_c && n3) {
        if (R.any_me)
            HIP_TRY(c, hipMemcpyAsync(R.bb.lag, lag_c, n3 * sizeof(double), kind, s));
        else
            HIP_TRY(c, hipMemsetAsync(R.bb.lag, 0, n3 * sizeof(double), s));
    }
    if (step >= 0) {
        R.step = step;
        const unsigned long long st64 = (unsigned long long)step;
        HIP_TRY(c, hipMemcpyAsync(R.d_step, &st64, sizeof(st64), hipMemcpyHostToDevice, s));
        // The cell-list heads carry the stamp of the step that wrote them.
        // After a rewind, heads written by the earlier pass over the same
        // step numbers would read as live; clear them all.
        if (R.cells.heads)
            HIP_TRY(c, hipMemsetAsync(R.cells.heads, 0,
                                      sizeof(unsigned long long) * (size_t)R.cells.n[0] * R.cells.n[1] * R.cells.n[2],
                                      s));
    }
    HIP_TRY(c, hipMemsetAsync(R.bb.flag, 0, sizeof(unsigned int), s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->error_state = false;
    return ICM_OK;
}

icm_status icm_step(icm_ctx* c, int64_t n_steps, uint32_t flags) {
    if (!c) return fail(nullptr, ICM_E_INVALID, "NULL context");
    if (c->error_state) return fail(c, ICM_E_STATE, "context is in an error state; call icm_set_state first");
    if (n_steps < 0) return fail(c, ICM_E_INVALID, "n_steps must be >= 0");
    if (flags & ~(uint32_t)ICM_STEP_GRAPH) return fail(c, ICM_E_INVALID, "unknown icm_step flags 0x%x", flags);
    hipStream_t s = c->stream;
    const bool graph = (flags & ICM_STEP_GRAPH) && !c->timing;
    if (graph && n_steps > 0 && !c->graph_exec) {
        icm_status st = capture_step(c);
        if (st != ICM_OK) return st;
    }
    for (int64_t n = 0; n < n_steps; ++n) {
        if (graph) {
            HIP_TRY(c, hipGraphLaunch(c->graph_exec, s));
        } else if (c->precision == ICM_FP64) {
            enqueue_all<double>(c, s);
        } else {
            enqueue_all<float>(c, s);
        }
    }
    for (Replica& R : c->reps) R.step += n_steps;
    HIP_TRY(c, hipGetLastError());
    unsigned int flag = 0;
    for (Replica& R : c->reps) {
        unsigned int f = 0;
        HIP_TRY(c, hipMemcpyAsync(&f, R.bb.flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        flag |= f;
    }
    if (c->timing) harvest_timing(c);
    if (flag) {
        c->error_state = true;
        return fail(c, ICM_E_NUMERIC, "numeric failure flag 0x%x (1: non-finite blob state, 2: blob moved > h)",
                    flag);
    }
    return ICM_OK;
}

icm_status icm_get_state(icm_ctx* c, int32_t replica, void* v, double* q, double* u, double* lag_c, icm_diag* d,
                         uint32_t flags) {
    icm_status st = check_replica(c, replica);
    if (st != ICM_OK) return st;
    Replica& R = c->reps[replica];
    const bool dev = (flags & ICM_PTRS_DEVICE) != 0;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t n3 = 3 * (size_t)R.nb;
    hipStream_t s = c->stream;
    if (v) HIP_TRY(c, hipMemcpyAsync(v, field_ptr(c, R), field_bytes(c, R), kind, s));
    if (q && n3) HIP_TRY(c, hipMemcpyAsync(q, R.bb.q, n3 * sizeof(double), kind, s));
    if (u && n3) HIP_TRY(c, hipMemcpyAsync(u, R.bb.u, n3 * sizeof(double), kind, s));
    if (lag_c && n3) HIP_TRY(c, hipMemcpyAsync(lag_c, R.bb.lag, n3 * sizeof(double), kind, s));
    if (d) {
        double acc[16];
        HIP_TRY(c, hipMemsetAsync(R.diag, 0, 16 * sizeof(double), s));
        if (c->precision == ICM_FP64)
            icm::launch_field_diag(R.gd, R.p.rho, R.diag, s);
        else
            icm::launch_field_diag(R.gf, R.p.rho, R.diag, s);
        icm::launch_blob_diag(R.nb, R.bb.me, R.bb.u, R.diag + 8, s);
        HIP_TRY(c, hipGetLastError());
        HIP_TRY(c, hipMemcpyAsync(acc, R.diag, sizeof(acc), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        for (int a = 0; a < 3; ++a) d->momentum[a] = acc[a] + acc[8 + a];
        if (R.gf.k0 && c->precision == ICM_FP32_GRID) {
            // the fluid's momentum is the carried FP64 mean velocity times rho V
            double k0[3];
            HIP_TRY(c, hipMemcpy(k0, R.gf.k0, sizeof(k0), hipMemcpyDeviceToHost));
            const double rv = R.p.rho * R.p.h * R.p.h * R.p.h * (double)R.gf.ncell;
            for (int a = 0; a < 3; ++a) d->momentum[a] = rv * k0[a] + acc[8 + a];
        }
        d->ke_fluid = acc[3];
        d->ke_blob = acc[11];
        d->max_div = acc[4] > 0 ? acc[5] / acc[4] : 0.0;
        d->max_alpha = R.p.dt / R.p.h * std::max(acc[4], acc[12]);
        d->step = R.step;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return ICM_OK;
}

icm_status icm_set_fft_shapes(icm_ctx* c, const icm_tune_result* shapes, int32_t count) {
    if (!c) return fail(nullptr, ICM_E_INVALID, "NULL context");
    if (count < 0 || (count > 0 && !shapes)) return fail(c, ICM_E_INVALID, "shapes must hold count entries");
    auto pow2 = [](int v) { return v >= 1 && v <= 64 && (v & (v - 1)) == 0; };
    for (int e = 0; e < count; ++e) {
        const icm_tune_result& r = shapes[e];
        if (!pow2(r.y_columns) || !pow2(r.z_columns) || (r.z_small_plan != 0 && r.z_small_plan != 1) ||
            !(r.x_threads == 64 || r.x_threads == 128 || r.x_threads == 256 || r.x_threads == 512) ||
            !(r.rhs_z_chunk == 0 || r.rhs_z_chunk == 4 || r.rhs_z_chunk == 8 || r.rhs_z_chunk == 16))
            return fail(c, ICM_E_INVALID, "entry %d: launch shape out of range", e);
        bool any = false;
        for (const Replica& R : c->reps)
            any = any || (R.p.n[0] == r.n[0] && R.p.n[1] == r.n[1] && R.p.n[2] == r.n[2]);
        if (!any) return fail(c, ICM_E_INVALID, "entry %d: no replica has grid %d x %d x %d", e, r.n[0], r.n[1], r.n[2]);
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int e = 0; e < count; ++e) {
        const icm_tune_result& r = shapes[e];
        for (Replica& R : c->reps) {
            if (R.p.n[0] != r.n[0] || R.p.n[1] != r.n[1] || R.p.n[2] != r.n[2]) continue;
            R.zc_tuned = r.rhs_z_chunk;
            auto apply = [&](auto& g) {
                g.By = r.y_columns;
                g.Bz = r.z_columns;
                g.zsmall = r.z_small_plan;
                g.xt = r.x_threads;
            };
            if (c->precision == ICM_FP64)
                apply(R.gd);
            else
                apply(R.gf);
        }
    }
    return sync_batches(c);
}

icm_status icm_get_advection_lag(icm_ctx* c, int32_t replica, void* lag, int32_t* valid, uint32_t flags) {
    icm_status st = check_replica(c, replica);
    if (st != ICM_OK) return st;
    Replica& R = c->reps[replica];
    unsigned int* hist = adv_hist_of(c, R);
    if (!hist) return fail(c, ICM_E_INVALID, "replica %d has advection off", replica);
    const bool dev = (flags & ICM_PTRS_DEVICE) != 0;
    hipStream_t s = c->stream;
    void* adv = c->precision == ICM_FP64 ? (void*)R.gd.adv : (void*)R.gf.adv;
    if (lag) HIP_TRY(c, hipMemcpyAsync(lag, adv, field_bytes(c, R), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    unsigned int h = 0;
    if (valid) HIP_TRY(c, hipMemcpyAsync(&h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    if (valid) *valid = h != 0u ? 1 : 0;
    return ICM_OK;
}

icm_status icm_set_advection_lag(icm_ctx* c, int32_t replica, const void* lag, uint32_t flags) {
    icm_status st = check_replica(c, replica);
    if (st != ICM_OK) return st;
    Replica& R = c->reps[replica];
    unsigned int* hist = adv_hist_of(c, R);
    if (!hist) return fail(c, ICM_E_INVALID, "replica %d has advection off", replica);
    const bool dev = (flags & ICM_PTRS_DEVICE) != 0;
    hipStream_t s = c->stream;
    void* adv = c->precision == ICM_FP64 ? (void*)R.gd.adv : (void*)R.gf.adv;
    const unsigned int one = 1u;
    if (lag) {
        HIP_TRY(c, hipMemcpyAsync(adv, lag, field_bytes(c, R), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(hist, &one, sizeof(one), hipMemcpyHostToDevice, s));
    } else {
        HIP_TRY(c, hipMemsetAsync(hist, 0, sizeof(unsigned int), s));
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return ICM_OK;
}

icm_status icm_autotune(icm_ctx* c, icm_tune_result* results, int32_t capacity, int32_t* n_results) {
    if (!c) return fail(nullptr, ICM_E_INVALID, "NULL context");
    if (c->error_state) return fail(c, ICM_E_STATE, "context is in an error state; call icm_set_state first");
    if (capacity < 0 || (capacity > 0 && !results)) return fail(c, ICM_E_INVALID, "results must hold capacity entries");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return c->precision == ICM_FP64 ? autotune_t<double>(c, results, capacity, n_results)
                                    : autotune_t<float>(c, results, capacity, n_results);
}

icm_status icm_set_timing(icm_ctx* c, int32_t enable) {
    if (!c) return fail(nullptr, ICM_E_INVALID, "NULL context");
    c->timing = enable != 0;
    return ICM_OK;
}

icm_status icm_get_timing(icm_ctx* c, icm_timing* out, int32_t reset) {
    if (!c || !out) return fail(c, ICM_E_INVALID, "NULL argument");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    harvest_timing(c);
    for (int i = 0; i < 16; ++i) {
        out->ms[i] = c->phase_ms[i];
        out->launches[i] = c->phase_n[i];
    }
    if (reset)
        for (int i = 0; i < 16; ++i) {
            c->phase_ms[i] = 0;
            c->phase_n[i] = 0;
        }
    return ICM_OK;
}

int32_t icm_num_blobs(const icm_ctx* c, int32_t replica) {
    if (!c || replica < 0 || replica >= (int32_t)c->reps.size()) return -1;
    return c->reps[replica].nb;
}

void icm_destroy(icm_ctx* c) {
    if (!c) return;
    if (c->stream || c->owns_ws) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipStream_t st : c->branch) (void)hipStreamDestroy(st);
    if (c->owns_ws && c->ws) (void)hipFree(c->ws);
    delete c;
}

const char* icm_last_error(const icm_ctx* c) { return c ? c->err.c_str() : g_last_error; }

}  // extern "C"

namespace icm {
icm_status fail_without_context(icm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}
}  // namespace icm

