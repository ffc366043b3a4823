// C ABI, plan management and the projected-CG driver.
//
// Projected CG on G K in strain space (Sec. "Compatibility projection": the
// test strains are projected by G, and gradient-based solvers started from a
// compatible field stay compatible) is run in its factored form: with
// e~ = B u the strain-space iterates are those of CG on K u = f preconditioned
// by M = B^T B, since G = B (B^T B)^+ B^T (small-strain appendix).  All Krylov
// vectors are nodal displacement fields; B, B^T run as real-space stencils
// (kern_stencil.hip) and only M^+ is applied per wavevector
// (kern_fft.hip).  Per iteration and load case:
//   stencil:  q = K p, p.q
//   scalars:  alpha = rho / p.q
//   FFT:      r -= alpha q fused into the last-axis r2c, first-axis pass with
//             z^ = M^-1 r^ and rho_new = r.z by Parseval
//   scalars:  stop test sqrt(rho_new / f.M^+f) <= tol, beta = rho_new / rho
//   FFT:      inverse passes; the last one applies u += alpha p, p = z + beta p
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "feh_internal.hpp"

namespace feh {

static thread_local std::string g_err;

int set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return FEH_OK;
    return set_error(FEH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Stockham passes for the radix sequence rad (product n).
static bool make_axis(int n, const std::vector<int> &rad, AxisFFT &ax) {
    if ((int)rad.size() > kMaxRadixCount) return false;
    ax = AxisFFT{};
    ax.n = n;
    int Lstar = 1;
    for (size_t s = 0; s < rad.size(); ++s) {
        PassInfo ps;
        ps.R = rad[s];
        ps.Lstar = Lstar;
        ps.m = FastDiv::make((uint32_t)(n / (Lstar * rad[s])));
        ax.pass[s] = ps;
        Lstar *= rad[s];
    }
    if (Lstar != n) return false;
    ax.npass = (int)rad.size();
    return true;
}

// Default factorisation: greedily the largest radices with butterflies
// (8, 4, 2, 3, 5, 7, 11, 13), then each remaining prime factor as one
// direct-DFT pass.
static bool default_radices(int n, std::vector<int> &rad) {
    rad.clear();
    int m = n;
    const int order[] = {8, 4, 2, 3, 5, 7, 11, 13};
    for (int r : order)
        while (m % r == 0 && m > 1) {
            rad.push_back(r);
            m /= r;
        }
    for (int f = 17; m > 1 && f * f <= m; f += 2)
        while (m % f == 0) {
            rad.push_back(f);
            m /= f;
        }
    if (m > 1) rad.push_back(m);  // the last prime factor
    return n >= 1;
}

static bool factorize(int n, AxisFFT &ax) {
    std::vector<int> rad;
    return default_radices(n, rad) && make_axis(n, rad, ax);
}

// Candidate radix sequences of the autotuner: the distinct orders of the
// default factorisation and of the one with the power-of-two part in
// radix-4 passes (at most 12).
static std::vector<std::vector<int>> radix_candidates(int n) {
    std::vector<std::vector<int>> out;
    auto add_orders = [&](std::vector<int> r) {
        std::sort(r.begin(), r.end());
        do {
            if (std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
        } while (out.size() < 12 && std::next_permutation(r.begin(), r.end()));
    };
    std::vector<int> d;
    if (!default_radices(n, d)) return out;
    out.push_back(d);  // the default first
    add_orders(d);
    int m = n, e = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++e;
    }
    std::vector<int> f;
    for (int i = 0; i < e / 2; ++i) f.push_back(4);
    if (e % 2) f.push_back(2);
    for (int r : d)
        if (r % 2) f.push_back(r);
    if (!f.empty()) add_orders(f);
    return out;
}

static void layout(feh_plan &p) {
    const size_t vec = (size_t)p.L * p.dim * p.N * p.rsize;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    p.off_u = take(vec);
    // r: a real field, or in the CG of cg_residual_spectral its last-axis half spectrum
    p.off_r = take(std::max(vec, (size_t)p.L * p.dim * p.Nspec * 2 * p.rsize));
    p.off_p = take(vec);
    p.off_q = take(vec);
    p.off_spec = take((size_t)p.L * p.dim * p.Nspec * 2 * p.rsize);
    p.off_lam = take(p.nbatch * p.N * p.rsize);
    p.off_mu = take(p.nbatch * p.N * p.rsize);
    for (int a = 0; a < 3; ++a) {
        const size_t na = (size_t)p.n[a];
        p.off_tw[a] = take(na * 2 * p.rsize);
        p.off_om[a] = take(na * 2 * sizeof(double));
        p.off_aa[a] = take(na * 2 * sizeof(double));
    }
    p.off_tab = take(kMaxPhase * 2 * sizeof(double));
    p.off_ebar = take((size_t)p.L * 9 * sizeof(double));
    p.off_sums = take((size_t)post_num_slots(p) * sizeof(double));
    // the autotuner may go down to a quarter of the default first-axis pencils
    const long long inner0 = p.dim == 3 ? p.n[1] * p.nh : p.nh;
    const int pbmin = std::max(1, first_pencils_default(p) / 4);
    int sp = stencil_num_parts(p);
    {
        // the most partial sums any stencil tile shape produces
        const int keep = p.tune_stencil_vy;
        p.tune_stencil_vy = 8;
        sp = std::max(sp, stencil_num_parts(p));
        p.tune_stencil_vy = keep;
    }
    const int fp = (int)((inner0 + pbmin - 1) / pbmin);
    p.part_stride = (size_t)(sp > fp ? sp : fp);
    size_t parts = p.part_stride * p.L;
    const size_t post_parts = (size_t)post_num_slots(p) * post_num_parts(p);
    if (post_parts > parts) parts = post_parts;
    p.off_part = take(parts * sizeof(double));
    p.off_state = take((size_t)p.L * sizeof(LcState));
    p.off_flag = take(256);
    // sensitivity pair list: l, m (int), group offsets (2 kMaxLoad ints, keeps the
    // weights 8-byte aligned), weights (double)
    p.off_pairs = take((size_t)kMaxLoad * (kMaxLoad + 1) / 2 * (2 * sizeof(int) + sizeof(double)) +
                       2 * kMaxLoad * sizeof(int));
    // (B^*B)^-1 per wavevector: D real diagonal + 3 (2D: 1) complex upper
    // entries, for whole pencil blocks (any block size up to 32)
    {
        const size_t ncomp = p.dim == 3 ? 9 : 4;
        p.off_minv = take(ncomp * (size_t)(inner0 + 32) * (size_t)p.n[0] * p.rsize);
    }
    p.total = o;
}

// e^{+2 pi i j / n} with the symmetries of the circle applied exactly: the
// angle is reduced to [0, pi/4] in integer arithmetic, so the table is exactly
// conjugate-symmetric and exact at multiples of pi/2.
static void cis_exact(long long j, long long n, double &c, double &s) {
    j %= n;
    if (j < 0) j += n;
    bool neg_s = false, neg_c = false;
    if (2 * j > n) {
        j = n - j;
        neg_s = true;
    }
    long long a = 2 * j, b = n;  // angle = pi a / b, a / b in [0, 1]
    if (2 * a > b) {
        a = b - a;               // pi - angle
        neg_c = true;
    }
    double cc, ss;
    if (4 * a > b) {             // pi/2 - pi u with u = (b - 2a) / (2b) in [0, 1/4)
        const double u = (double)(b - 2 * a) / (double)(2 * b);
        cc = std::sin(M_PI * u);
        ss = std::cos(M_PI * u);
    } else {
        const double t = (double)a / (double)b;
        cc = std::cos(M_PI * t);
        ss = std::sin(M_PI * t);
    }
    c = neg_c ? -cc : cc;
    s = neg_s ? -ss : ss;
}

static void tables(feh_plan &p) {
    for (int a = 0; a < 3; ++a) {
        const int n = (int)p.n[a];
        p.tw_host[a].assign(2 * n, 0.0);
        p.om_host[a].assign(2 * n, 0.0);
        p.aa_host[a].assign(2 * n, 0.0);
        for (int j = 0; j < n; ++j) {
            double c, s, ch, sh;
            cis_exact(j, n, c, s);
            cis_exact(j, 2 * (long long)n, ch, sh);  // half angle
            // twiddle exp(-i th), th = 2 pi j / n
            p.tw_host[a][2 * j] = c;
            p.tw_host[a][2 * j + 1] = -s;
            // omega = exp(+i th); a = (omega - 1)/h = (-2 sin^2(th/2) + i sin th)/h
            p.om_host[a][2 * j] = c;
            p.om_host[a][2 * j + 1] = s;
            p.aa_host[a][2 * j] = -2.0 * sh * sh / p.h[a];
            p.aa_host[a][2 * j + 1] = s / p.h[a];
        }
    }
}

static int upload_tables(feh_plan &p) {
    for (int a = 0; a < 3; ++a) {
        const int n = (int)p.n[a];
        if (p.prec == FEH_FP64) {
            CK(hip_check(hipMemcpyAsync(p.ws + p.off_tw[a], p.tw_host[a].data(), 2 * n * sizeof(double),
                                        hipMemcpyHostToDevice, p.stream),
                         "upload twiddles"));
        } else {
            std::vector<float> f(2 * n);
            for (int j = 0; j < 2 * n; ++j) f[j] = (float)p.tw_host[a][j];
            CK(hip_check(hipMemcpyAsync(p.ws + p.off_tw[a], f.data(), 2 * n * sizeof(float), hipMemcpyHostToDevice,
                                        p.stream),
                         "upload twiddles"));
            CK(hip_check(hipStreamSynchronize(p.stream), "upload twiddles"));
        }
        CK(hip_check(hipMemcpyAsync(p.ws + p.off_om[a], p.om_host[a].data(), 2 * n * sizeof(double),
                                    hipMemcpyHostToDevice, p.stream),
                     "upload phases"));
        CK(hip_check(hipMemcpyAsync(p.ws + p.off_aa[a], p.aa_host[a].data(), 2 * n * sizeof(double),
                                    hipMemcpyHostToDevice, p.stream),
                     "upload phases"));
    }
    return hip_check(hipStreamSynchronize(p.stream), "upload tables");
}

static int check_plan(const feh_plan *p, bool need_material) {
    if (!p) return set_error(FEH_EINVAL, "null plan");
    if (!p->ws) return set_error(FEH_ENOMEM, "workspace not set (feh_plan_set_workspace)");
    if (need_material && !p->material_set) return set_error(FEH_EINVAL, "material not set");
    return FEH_OK;
}

static int read_flag(feh_plan &p, int *flag_dev, const char *what) {
    int h = 0;
    CK(hip_check(hipMemcpyAsync(&h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, p.stream), what));
    CK(hip_check(hipStreamSynchronize(p.stream), what));
    return h ? set_error(FEH_EINVAL, std::string(what) + ": invalid material value") : FEH_OK;
}

// z = M^+ r on SoA fields (spectrum buffer as scratch); Parseval r.z partials.
// r is consumed by the first pass, so z may be the same buffer.
// z = M^+ r.  rhat non-null (3D): the last-axis half spectrum of r is written
// there and kept (the forward middle pass reads it into the spectrum).
static int precondition(const feh_plan &p, const void *r, void *z, double *partial, const LcState *st,
                        bool unit_volume, void *rhat = nullptr) {
    FftArgs fa;
    fa.unit_volume = unit_volume;
    fa.r = r;
    fa.spec = rhat ? rhat : p.ws + p.off_spec;
    fa.z = z;
    fa.partial = partial;
    fa.state = st;
    fa.out_scale = 1.0 / (double)p.N;
    CK(launch_forward_last(p, fa));
    fa.spec = p.ws + p.off_spec;
    if (p.dim == 3) {
        FftArgs fm = fa;
        fm.spec_in = rhat;
        CK(launch_middle(p, fm, false));
        CK(launch_first_fused(p, fa));
    } else {
        FftArgs ff = fa;
        ff.spec_in = rhat;
        CK(launch_first_fused(p, ff));
    }
    if (p.dim == 3) CK(launch_middle(p, fa, true));
    return launch_inverse_last(p, fa);
}

// Optional event timing of the CG loop: a (start, end) event pair around
// every launch, drained after each host synchronisation.
struct ProfScope {
    const feh_plan &p;
    int kind;
    ProfScope(const feh_plan &pl, int k) : p(pl), kind(k) {
        if (!p.prof_on) return;
        if (2 * p.prof_used + 2 > p.prof_ev.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
            p.prof_ev.push_back(a);
            p.prof_ev.push_back(b);
            p.prof_kind.push_back(0);
        }
        (void)hipEventRecord(p.prof_ev[2 * p.prof_used], p.stream);
    }
    ~ProfScope() {
        if (!p.prof_on || 2 * p.prof_used + 2 > p.prof_ev.size()) return;
        (void)hipEventRecord(p.prof_ev[2 * p.prof_used + 1], p.stream);
        p.prof_kind[p.prof_used] = kind;
        ++p.prof_used;
    }
};

static void prof_drain(const feh_plan &p) {
    for (size_t i = 0; i < p.prof_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.prof_ev[2 * i], p.prof_ev[2 * i + 1]) == hipSuccess) {
            p.prof_ms[p.prof_kind[i]] += ms;
            p.prof_n[p.prof_kind[i]] += 1;
        }
    }
    p.prof_used = 0;
}

// One preconditioned CG iteration for every active load case:
//   q = K p, alpha = rho / p.q; r -= alpha q and z = M^+ r (FFT pipeline, with
//   rho_new = r.z from the k-solve); beta = rho_new / rho; then, fused into the
//   last inverse pass, u += alpha p and p = z + beta p.  A load case that stops
//   at the convergence test keeps its last u += alpha p pending (applied by
//   the finalisation).
static int cg_iteration(const feh_plan &p, LcState *st, double tol, int max_iter) {
    double *part = p.ptr<double>(p.off_part);
    StencilArgs sa;
    sa.in0 = p.ws + p.off_p;
    sa.out0 = p.ws + p.off_q;
    sa.partial = part;
    sa.state = st;
    sa.unit_volume = true;
    {
        ProfScope ps(p, 0);
        CK(launch_stencil(p, ST_CG, sa));
    }
    {
        ProfScope ps(p, 1);
        CK(launch_finish_pq(p, st, part, stencil_num_parts(p)));
    }
    FftArgs fa;
    fa.r = p.ws + p.off_r;
    fa.q = p.ws + p.off_q;
    fa.r_out = p.ws + p.off_r;
    fa.spec = p.ws + p.off_spec;
    fa.p_upd = p.ws + p.off_p;
    fa.u_upd = p.ws + p.off_u;
    fa.partial = part;
    fa.state = st;
    fa.out_scale = 1.0 / (double)p.N;
    fa.unit_volume = true;
    // residual kept as a last-axis half spectrum r^: the forward last pass
    // transforms q and updates r^ -= alpha q^ in place (the FFT is linear),
    // and the next forward pass (middle in 3D, first axis in 2D) reads r^
    // into the spectrum
    const bool rs = cg_residual_spectral(p);
    {
        ProfScope ps(p, 2);
        FftArgs fl = fa;
        if (rs) {
            fl.r = nullptr;
            fl.r_out = nullptr;
            fl.spec = p.ws + p.off_r;
            fl.rspec = true;
        }
        CK(launch_forward_last(p, fl));
    }
    if (p.dim == 3) {
        ProfScope ps(p, 3);
        FftArgs fm = fa;
        if (rs) fm.spec_in = p.ws + p.off_r;
        CK(launch_middle(p, fm, false));
    }
    {
        ProfScope ps(p, 4);
        FftArgs ff = fa;
        if (rs && p.dim == 2) ff.spec_in = p.ws + p.off_r;  // 2D: the first-axis pass reads r^
        CK(launch_first_fused(p, ff));
    }
    {
        ProfScope ps(p, 7);
        CK(launch_finish_rho(p, st, part, first_num_parts(p), 2, tol, max_iter));
    }
    if (p.dim == 3) {
        ProfScope ps(p, 5);
        CK(launch_middle(p, fa, true));
    }
    ProfScope ps(p, 6);
    return launch_inverse_last(p, fa);
}

static void invert(int n, std::vector<double> &A, bool &ok) {
    // Gauss-Jordan with partial pivoting, in place (row-major n x n)
    std::vector<double> I(n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    ok = true;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (std::fabs(A[piv * n + c]) < 1e-300) {
            ok = false;
            return;
        }
        for (int k = 0; k < n; ++k) {
            std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(I[c * n + k], I[piv * n + k]);
        }
        const double d = 1.0 / A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] *= d;
            I[c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                I[r * n + k] -= f * I[c * n + k];
            }
        }
    }
    A = I;
}

// Workspace of feh_solve_noalloc: a file-scope device array (every GPU the
// library runs on holds its own copy until the process ends).  In host code
// `scratch` is only a stand-in for the symbol: its device address is queried
// once per device, with that device current, and used everywhere instead.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device of `stream`.
static int static_scratch(hipStream_t stream, char **out) {
    int dev = 0;
    CK(hip_check(hipStreamGetDevice(stream, &dev), "device of the plan's stream"));
    if (dev < 0 || dev >= kMaxDevices) return set_error(FEH_ENOTSUP, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        CK(hip_check(hipGetDevice(&cur), "current device"));
        if (cur != dev) CK(hip_check(hipSetDevice(dev), "select the plan's device"));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        CK(hip_check(e, "address of the static scratch"));
        if (!ptr) return set_error(FEH_EHIP, "null address of the static scratch");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return FEH_OK;
}

}  // namespace feh

using namespace feh;

extern "C" {

const char *feh_last_error(void) { return g_err.c_str(); }

int feh_version(void) { return 10000; }

static int plan_create(feh_plan **plan, int dim, const int64_t n[], const double h[], int n_batch, int n_load,
                       int precision, void *hip_stream) {
    try {
        if (!plan) return set_error(FEH_EINVAL, "null plan pointer");
        *plan = nullptr;
        if (dim != 2 && dim != 3) return set_error(FEH_EINVAL, "dim must be 2 or 3");
        if (!n) return set_error(FEH_EINVAL, "null size array");
        if (n_batch < 1 || n_load < 1 || (long long)n_batch * n_load > kMaxLoad)
            return set_error(FEH_EINVAL, "n_batch * n_load must be in [1, 64]");
        if (precision != FEH_FP64 && precision != FEH_FP32) return set_error(FEH_EINVAL, "bad precision");
        auto p = new feh_plan();
        p->dim = dim;
        p->nbatch = n_batch;
        p->G = n_load;
        p->L = n_batch * n_load;
        p->prec = precision;
        p->rsize = precision == FEH_FP64 ? 8 : 4;
        p->stream = static_cast<hipStream_t>(hip_stream);
        p->N = 1;
        for (int a = 0; a < dim; ++a) {
            if (n[a] < 2 || n[a] > kMaxN) {
                delete p;
                return set_error(FEH_EINVAL, "grid sizes must lie in [2, 4096]");
            }
            p->n[a] = n[a];
            p->h[a] = h ? h[a] : 1.0;
            if (!(p->h[a] > 0.0) || !std::isfinite(p->h[a])) {
                delete p;
                return set_error(FEH_EINVAL, "voxel sizes must be positive and finite");
            }
            p->N *= n[a];
        }
        if (p->N > (int64_t(1) << 31)) {
            delete p;
            return set_error(FEH_EINVAL, "grid too large (N > 2^31)");
        }
        const int64_t nl = n[dim - 1];
        p->last_even = (nl % 2) == 0;
        p->nh = nl / 2 + 1;
        p->Nspec = p->N / nl * p->nh;
        p->ne = dim == 3 ? 6 : 2;
        for (int a = 0; a < dim; ++a) {
            int len = (int)n[a];
            if (a == dim - 1 && p->last_even) len /= 2;
            if (!factorize(len, p->fft[a])) {
                delete p;
                return set_error(FEH_ENOTSUP, "grid size needs more FFT passes than supported");
            }
        }
        // LDS capacity of the transforms (points per workgroup)
        const int cap = (precision == FEH_FP32 ? 24 : 16) * 256;
        const int nc = p->fft[dim - 1].n;
        if (nc * dim > cap || (int)n[0] * dim > cap || (dim == 3 && (int)n[1] > cap)) {
            delete p;
            return set_error(FEH_ENOTSUP, "axis too long for the LDS-staged transform");
        }
        tables(*p);
        layout(*p);
        *plan = p;
        return FEH_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_plan_create(feh_plan **plan, int dim, const int64_t n[], const double h[], int n_load, int precision,
                    void *hip_stream) {
    return plan_create(plan, dim, n, h, 1, n_load, precision, hip_stream);
}

int feh_plan_create_batch(feh_plan **plan, int dim, const int64_t n[], const double h[], int n_batch, int n_load,
                          int precision, void *hip_stream) {
    return plan_create(plan, dim, n, h, n_batch, n_load, precision, hip_stream);
}

int feh_plan_destroy(feh_plan *plan) {
    if (plan)
        for (hipEvent_t e : plan->prof_ev) (void)hipEventDestroy(e);
    delete plan;
    return FEH_OK;
}

int feh_plan_workspace_bytes(const feh_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return set_error(FEH_EINVAL, "null argument");
    *bytes = plan->total;
    return FEH_OK;
}

int feh_plan_set_workspace(feh_plan *plan, void *dev_ptr, size_t bytes) {
    try {
        if (!plan || !dev_ptr) return set_error(FEH_EINVAL, "null argument");
        if (bytes < plan->total) return set_error(FEH_ENOMEM, "workspace too small");
        if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return set_error(FEH_EINVAL, "workspace must be 256-byte aligned");
        plan->ws = static_cast<char *>(dev_ptr);
        plan->ws_bytes = bytes;
        plan->material_set = false;
        plan->solved = false;
        plan->field_nu = -2.0;
        return upload_tables(*plan);
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_set_material_lame(feh_plan *plan, const void *lambda_dev, const void *mu_dev) {
    CK(check_plan(plan, false));
    if (!lambda_dev || !mu_dev) return set_error(FEH_EINVAL, "null material pointer");
    int *flag = plan->ptr<int>(plan->off_flag);
    CK(launch_fill(*plan, flag, 1, 0.0));  // a kernel, not a memset node (capturable)
    plan->material_set = false;
    plan->solved = false;
    plan->field_nu = -2.0;
    CK(launch_material_lame(*plan, lambda_dev, mu_dev, flag));
    CK(read_flag(*plan, flag, "feh_set_material_lame"));
    plan->material_set = true;
    plan->solved = false;
    return FEH_OK;
}

int feh_set_material_phases(feh_plan *plan, const int32_t *phase_dev, const double *E_nu_host, int n_phase) {
    CK(check_plan(plan, false));
    if (!phase_dev || !E_nu_host) return set_error(FEH_EINVAL, "null material pointer");
    if (n_phase < 1 || n_phase > kMaxPhase) return set_error(FEH_EINVAL, "n_phase must be in [1, 4096]");
    std::vector<double> tab(2 * n_phase);
    for (int k = 0; k < n_phase; ++k) {
        const double E = E_nu_host[2 * k], nu = E_nu_host[2 * k + 1];
        if (!std::isfinite(E) || E < 0.0 || !(nu > -1.0 && nu < 0.5))
            return set_error(FEH_EINVAL, "phase table needs E >= 0 and -1 < nu < 0.5");
        tab[2 * k] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        tab[2 * k + 1] = E / (2.0 * (1.0 + nu));
    }
    double *dtab = plan->ptr<double>(plan->off_tab);
    CK(hip_check(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, plan->stream),
                 "phase table"));
    int *flag = plan->ptr<int>(plan->off_flag);
    CK(launch_fill(*plan, flag, 1, 0.0));  // a kernel, not a memset node (capturable)
    plan->material_set = false;
    plan->solved = false;
    plan->field_nu = -2.0;
    CK(launch_material_phases(*plan, phase_dev, dtab, n_phase, flag));
    CK(read_flag(*plan, flag, "feh_set_material_phases"));
    plan->material_set = true;
    plan->solved = false;
    return FEH_OK;
}

int feh_set_material_field(feh_plan *plan, const void *E_dev, double nu) {
    CK(check_plan(plan, false));
    if (!E_dev) return set_error(FEH_EINVAL, "null material pointer");
    if (!(nu > -1.0 && nu < 0.5)) return set_error(FEH_EINVAL, "nu must lie in (-1, 0.5)");
    int *flag = plan->ptr<int>(plan->off_flag);
    CK(launch_fill(*plan, flag, 1, 0.0));  // a kernel, not a memset node (capturable)
    plan->material_set = false;
    plan->solved = false;
    plan->field_nu = -2.0;
    CK(launch_material_field(*plan, E_dev, nu, flag));
    CK(read_flag(*plan, flag, "feh_set_material_field"));
    plan->material_set = true;
    plan->field_nu = nu;
    plan->solved = false;
    return FEH_OK;
}

// ---------------------------------------------------------------------------
// solve stages: set-up (right-hand side, first search direction), CG loop,
// finalisation (pending u update, post-processing, host outputs)
// ---------------------------------------------------------------------------
static int solve_begin(feh_plan &p, const double *Ebar_host, double tol, int max_iter, const void *u0_dev) {
    if (!Ebar_host) return set_error(FEH_EINVAL, "null Ebar");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(FEH_EINVAL, "tol must be finite and >= 0");
    p.solved = false;
    if (max_iter < 1) return set_error(FEH_EINVAL, "max_iter must be >= 1");
    const int D = p.dim;
    for (int l = 0; l < p.L; ++l)
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                const double a = Ebar_host[(l * D + i) * D + j], b = Ebar_host[(l * D + j) * D + i];
                if (!std::isfinite(a)) return set_error(FEH_EINVAL, "Ebar must be finite");
                if (std::fabs(a - b) > 1e-12 * (std::fabs(a) + std::fabs(b)) + 1e-300)
                    return set_error(FEH_EINVAL, "Ebar must be symmetric");
            }
    // the kernels read D x D per load case
    std::vector<double> eb(Ebar_host, Ebar_host + (size_t)p.L * D * D);
    double *ebar_dev = p.ptr<double>(p.off_ebar);
    CK(hip_check(hipMemcpyAsync(ebar_dev, eb.data(), eb.size() * sizeof(double), hipMemcpyHostToDevice, p.stream),
                 "upload Ebar"));
    // the host vector must outlive the asynchronous copy
    CK(hip_check(hipStreamSynchronize(p.stream), "upload Ebar"));
    LcState *st = p.ptr<LcState>(p.off_state);
    double *part = p.ptr<double>(p.off_part);
    const size_t nvec = (size_t)p.L * D * p.N;
    CK(launch_init_state(p, st, p.L));
    StencilArgs sa;
    sa.Ebar = ebar_dev;
    sa.unit_volume = true;
    if (u0_dev) {
        CK(launch_aos_to_soa(p, u0_dev, p.ws + p.off_u));
        // the fluctuation is fixed up to a rigid translation: start from zero mean
        CK(launch_remove_mean(p, p.ws + p.off_u, part, p.ptr<double>(p.off_sums)));
        // reference f.M^+f from the right-hand side alone
        sa.in0 = nullptr;
        sa.out0 = p.ws + p.off_q;
        CK(launch_stencil(p, ST_RESID, sa));
        CK(precondition(p, p.ws + p.off_q, p.ws + p.off_q, part, nullptr, true));
        CK(launch_finish_rho(p, st, part, first_num_parts(p), 0, tol, max_iter));
        sa.in0 = p.ws + p.off_u;
    } else {
        CK(launch_fill(p, p.ws + p.off_u, nvec, 0.0));
        sa.in0 = nullptr;
    }
    // r = f - K u0, first search direction p = M^+ r; with the residual kept
    // as a last-axis half spectrum, r goes through q and its spectrum to r's place
    const bool rs = cg_residual_spectral(p);
    sa.out0 = p.ws + (rs ? p.off_q : p.off_r);
    CK(launch_stencil(p, ST_RESID, sa));
    CK(precondition(p, sa.out0, p.ws + p.off_p, part, nullptr, true, rs ? p.ws + p.off_r : nullptr));
    return launch_finish_rho(p, st, part, first_num_parts(p), u0_dev ? 1 : 11, tol, max_iter);
}

static int solve_end(feh_plan &p, void *u_dev, void *strain_dev, void *stress_dev, double *stress_mean_host,
                     double *energy_host, feh_report *report_host) {
    const int D = p.dim;
    LcState *st = p.ptr<LcState>(p.off_state);
    double *part = p.ptr<double>(p.off_part);
    CK(launch_finalize_u(p, p.ws + p.off_u, p.ws + p.off_p, st));
    double *sums = p.ptr<double>(p.off_sums);
    CK(launch_post_sums(p, p.ws + p.off_u, p.ptr<double>(p.off_ebar), strain_dev, stress_dev, part, sums));
    if (u_dev) CK(launch_soa_to_aos(p, p.ws + p.off_u, u_dev));
    const int ns = D == 3 ? 6 : 3;
    std::vector<double> hsum(post_num_slots(p));
    std::vector<LcState> hs(p.L);
    CK(hip_check(hipMemcpyAsync(hsum.data(), sums, hsum.size() * sizeof(double), hipMemcpyDeviceToHost, p.stream),
                 "read sums"));
    CK(hip_check(hipMemcpyAsync(hs.data(), st, p.L * sizeof(LcState), hipMemcpyDeviceToHost, p.stream),
                 "read CG state"));
    CK(hip_check(hipStreamSynchronize(p.stream), "solve"));
    if (stress_mean_host) {
        for (int l = 0; l < p.L; ++l) {
            const double *s = hsum.data() + l * ns;
            double *o = stress_mean_host + (size_t)l * D * D;
            if (D == 3) {
                const double full[9] = {s[0], s[5], s[4], s[5], s[1], s[3], s[4], s[3], s[2]};
                std::memcpy(o, full, sizeof(full));
            } else {
                const double full[4] = {s[0], s[2], s[2], s[1]};
                std::memcpy(o, full, sizeof(full));
            }
        }
    }
    if (energy_host) {
        // pairs within each microstructure; load cases of different
        // microstructures do not interact (zero)
        std::fill(energy_host, energy_host + (size_t)p.L * p.L, 0.0);
        int k = 0;
        for (int b = 0; b < p.nbatch; ++b)
            for (int li = 0; li < p.G; ++li)
                for (int mi = li; mi < p.G; ++mi, ++k) {
                    const int l = b * p.G + li, m = b * p.G + mi;
                    const double w = hsum[(size_t)p.L * ns + k];
                    energy_host[l * p.L + m] = w;
                    energy_host[m * p.L + l] = w;
                }
    }
    int rc = FEH_OK;
    for (int l = 0; l < p.L; ++l) {
        if (report_host) {
            report_host[l].iterations = hs[l].iters;
            report_host[l].status = hs[l].status;
            report_host[l].rel_residual = hs[l].relres;
        }
        if (hs[l].status == FEH_EBREAKDOWN) rc = FEH_EBREAKDOWN;
        else if ((hs[l].status == FEH_ENOCONV || hs[l].active) && rc == FEH_OK) rc = FEH_ENOCONV;
    }
    p.solved = rc != FEH_EBREAKDOWN;
    if (rc == FEH_ENOCONV) return set_error(rc, "max_iter reached before the tolerance");
    if (rc == FEH_EBREAKDOWN) return set_error(rc, "CG breakdown (p.q <= 0 or not finite)");
    return FEH_OK;
}

// Copy the CG states of the plans to the host (one synchronisation); true if
// any load case is still iterating.
static int any_active(feh_plan *const *plans, int n, std::vector<std::vector<LcState>> &hs, bool &any) {
    for (int i = 0; i < n; ++i) {
        feh_plan &p = *plans[i];
        hs[i].resize(p.L);
        CK(hip_check(hipMemcpyAsync(hs[i].data(), p.ptr<LcState>(p.off_state), p.L * sizeof(LcState),
                                    hipMemcpyDeviceToHost, p.stream),
                     "read CG state"));
    }
    for (int i = 0; i < n; ++i) CK(hip_check(hipStreamSynchronize(plans[i]->stream), "CG"));
    any = false;
    for (int i = 0; i < n; ++i)
        for (const LcState &s : hs[i]) any = any || s.active;
    return FEH_OK;
}

// The whole solve on the plan's current workspace: set-up, CG loop (host
// checks of the stop flags after chunks of 4, 8, then 16 iterations), and
// finalisation.
static int solve_all(feh_plan &p, const double *Ebar_host, double tol, int max_iter, const void *u0_dev, void *u_dev,
                     void *strain_dev, void *stress_dev, double *stress_mean_host, double *energy_host,
                     feh_report *report_host) {
    CK(solve_begin(p, Ebar_host, tol, max_iter, u0_dev));
    LcState *st = p.ptr<LcState>(p.off_state);
    std::vector<std::vector<LcState>> hs(1);
    feh_plan *pp = &p;
    int done = 0, chunk = 4;
    while (done < max_iter) {
        bool any = false;
        CK(any_active(&pp, 1, hs, any));
        prof_drain(p);
        if (!any) break;
        const int c = chunk < max_iter - done ? chunk : max_iter - done;
        for (int i = 0; i < c; ++i) CK(cg_iteration(p, st, tol, max_iter));
        done += c;
        if (chunk < 16) chunk *= 2;
    }
    return solve_end(p, u_dev, strain_dev, stress_dev, stress_mean_host, energy_host, report_host);
}

int feh_solve(feh_plan *plan, const double *Ebar_host, double tol, int max_iter, const void *u0_dev, void *u_dev,
              void *strain_dev, void *stress_dev, double *stress_mean_host, double *energy_host,
              feh_report *report_host) {
    try {
        const double t0 = wall_seconds();
        CK(check_plan(plan, true));
        feh_plan &p = *plan;
        const int rc = solve_all(p, Ebar_host, tol, max_iter, u0_dev, u_dev, strain_dev, stress_dev, stress_mean_host,
                                 energy_host, report_host);
        if (rc == FEH_OK || rc == FEH_ENOCONV || rc == FEH_EBREAKDOWN) stamp_reports(report_host, p.L, t0);
        return rc;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

// ---------------------------------------------------------------------------
// batches of plans: per stream, one HIP graph per chunk of CG iterations of
// the plans on that stream
// ---------------------------------------------------------------------------

struct feh_batch {
    std::vector<feh_plan *> plans;
    std::vector<hipStream_t> streams;    // the plans' distinct streams, first plan's first
    // instantiated graphs, keyed by (stream, chunk length, tol, max_iter): the
    // CG kernels read their state from device memory, so a graph replays for
    // as long as the plans, their workspaces and the stopping rule are unchanged
    struct Entry {
        int si;
        int chunk;
        double tol;
        int max_iter;
        hipGraphExec_t exec;
    };
    std::vector<Entry> graphs;
    int launches = 0;  // chunks run by graph launches in the last solve (for tests)
    // the plans' CG states copied back after each chunk (pinned, so the copy
    // is asynchronous), with one event per stream marking its copies
    LcState *hstate = nullptr;
    std::vector<size_t> hstate_at;       // first state of each plan in hstate
    std::vector<hipEvent_t> copied;
};

static void batch_clear(feh_batch &b) {
    for (auto &e : b.graphs) (void)hipGraphExecDestroy(e.exec);
    b.graphs.clear();
}

static void batch_release(feh_batch &b) {
    // a solve that ended on an error may have left state copies queued
    for (hipStream_t s : b.streams) (void)hipStreamSynchronize(s);
    batch_clear(b);
    for (hipEvent_t e : b.copied) (void)hipEventDestroy(e);
    b.copied.clear();
    if (b.hstate) (void)hipHostFree(b.hstate);
    b.hstate = nullptr;
}

// The graph of `chunk` CG iterations of the plans on stream si, captured on
// that stream (each stream's chain is a graph of its own, so the streams'
// graphs run concurrently as their eager launches do).
static int batch_graph(feh_batch &b, int si, int chunk, double tol, int max_iter, hipGraphExec_t &exec) {
    for (auto &e : b.graphs)
        if (e.si == si && e.chunk == chunk && e.tol == tol && e.max_iter == max_iter) {
            exec = e.exec;
            return FEH_OK;
        }
    hipStream_t s = b.streams[si];
    CK(hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture"));
    int rc = FEH_OK;
    for (int i = 0; i < chunk && rc == FEH_OK; ++i)
        for (feh_plan *p : b.plans) {
            if (p->stream != s) continue;
            rc = cg_iteration(*p, p->ptr<LcState>(p->off_state), tol, max_iter);
            if (rc != FEH_OK) break;
        }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);  // always end the capture, also after an error
    if (rc != FEH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    CK(hip_check(ec, "end capture"));
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK(hip_check(ei, "instantiate graph"));
    b.graphs.push_back({si, chunk, tol, max_iter, exec});
    return FEH_OK;
}

int feh_batch_create(feh_batch **out, feh_plan *const *plans, int n_plans) {
    try {
        if (!out) return set_error(FEH_EINVAL, "null batch pointer");
        *out = nullptr;
        if (!plans || n_plans < 1) return set_error(FEH_EINVAL, "need at least one plan");
        for (int i = 0; i < n_plans; ++i) {
            if (!plans[i]) return set_error(FEH_EINVAL, "null plan");
            if (plans[i]->stream == nullptr) return set_error(FEH_EINVAL, "a batch needs created (non-null) streams");
            for (int j = 0; j < i; ++j)
                if (plans[j] == plans[i]) return set_error(FEH_EINVAL, "a plan appears twice");
        }
        auto b = new feh_batch();
        b->plans.assign(plans, plans + n_plans);
        for (int i = 0; i < n_plans; ++i)
            if (std::find(b->streams.begin(), b->streams.end(), plans[i]->stream) == b->streams.end())
                b->streams.push_back(plans[i]->stream);
        size_t nst = 0;
        for (int i = 0; i < n_plans; ++i) {
            b->hstate_at.push_back(nst);
            nst += (size_t)plans[i]->L;
        }
        int rc = hip_check(hipHostMalloc(reinterpret_cast<void **>(&b->hstate), nst * sizeof(LcState)), "pinned CG states");
        for (size_t si = 0; si < b->streams.size() && rc == FEH_OK; ++si) {
            hipEvent_t e = nullptr;
            rc = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
            if (rc == FEH_OK) b->copied.push_back(e);
        }
        if (rc != FEH_OK) {
            batch_release(*b);
            delete b;
            return rc;
        }
        *out = b;
        return FEH_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    }
}

int feh_batch_destroy(feh_batch *b) {
    if (!b) return FEH_OK;
    batch_release(*b);
    delete b;
    return FEH_OK;
}

int feh_batch_solve(feh_batch *b, const double *const *Ebar_host, double tol, int max_iter, int use_graph,
                    double *const *stress_mean_host, double *const *energy_host, feh_report *const *report_host) {
    try {
        const double t0 = wall_seconds();
        if (!b) return set_error(FEH_EINVAL, "null batch");
        if (!Ebar_host) return set_error(FEH_EINVAL, "null Ebar table");
        const int n = (int)b->plans.size();
        for (int i = 0; i < n; ++i) {
            CK(check_plan(b->plans[i], true));
            if (b->plans[i]->prof_on) return set_error(FEH_EINVAL, "profiling is not available in a batch");
        }
        for (int i = 0; i < n; ++i) CK(solve_begin(*b->plans[i], Ebar_host[i], tol, max_iter, nullptr));
        int done = 0, chunk = 4;
        b->launches = 0;
        auto launch_chunk = [&](int c) -> int {
            if (use_graph) {
                for (int si = 0; si < (int)b->streams.size(); ++si) {
                    hipGraphExec_t exec = nullptr;
                    CK(batch_graph(*b, si, c, tol, max_iter, exec));
                    CK(hip_check(hipGraphLaunch(exec, b->streams[si]), "graph launch"));
                }
            } else {
                for (int it = 0; it < c; ++it)
                    for (feh_plan *p : b->plans) CK(cg_iteration(*p, p->ptr<LcState>(p->off_state), tol, max_iter));
            }
            ++b->launches;
            done += c;
            if (chunk < 8) chunk *= 2;  // the checks cost no idle time here, so short chunks
            return FEH_OK;
        };
        // states after the chunks launched so far, copied on each stream
        auto copy_states = [&]() -> int {
            for (int i = 0; i < n; ++i) {
                feh_plan &p = *b->plans[i];
                CK(hip_check(hipMemcpyAsync(b->hstate + b->hstate_at[i], p.ptr<LcState>(p.off_state), p.L * sizeof(LcState),
                                            hipMemcpyDeviceToHost, p.stream),
                             "read CG state"));
            }
            for (size_t si = 0; si < b->streams.size(); ++si)
                CK(hip_check(hipEventRecord(b->copied[si], b->streams[si]), "record"));
            return FEH_OK;
        };
        auto states_active = [&](bool &any) -> int {
            for (size_t si = 0; si < b->streams.size(); ++si) CK(hip_check(hipEventSynchronize(b->copied[si]), "CG"));
            any = false;
            for (int i = 0; i < n; ++i)
                for (int l = 0; l < b->plans[i]->L; ++l) any = any || b->hstate[b->hstate_at[i] + l].active;
            return FEH_OK;
        };
        // Stop checks one chunk behind: the next chunk is queued before the
        // host looks at the states after the previous one, so the streams do
        // not idle while it does; once every load case has stopped, the
        // chunk queued meanwhile runs kernels that return at once.
        bool any = false;
        CK(copy_states());
        CK(states_active(any));
        if (any && done < max_iter) {
            CK(launch_chunk(chunk < max_iter - done ? chunk : max_iter - done));
            CK(copy_states());
            while (done < max_iter) {
                CK(launch_chunk(chunk < max_iter - done ? chunk : max_iter - done));
                CK(states_active(any));
                if (!any) break;
                CK(copy_states());
            }
        }
        int rc = FEH_OK;
        for (int i = 0; i < n; ++i) {
            const int r = solve_end(*b->plans[i], nullptr, nullptr, nullptr, stress_mean_host ? stress_mean_host[i] : nullptr,
                                    energy_host ? energy_host[i] : nullptr, report_host ? report_host[i] : nullptr);
            if (r == FEH_EBREAKDOWN || (r != FEH_OK && rc == FEH_OK)) rc = r;
        }
        if (report_host)
            for (int i = 0; i < n; ++i) stamp_reports(report_host[i], b->plans[i]->L, t0);
        if (rc == FEH_ENOCONV) return set_error(rc, "max_iter reached before the tolerance (some plan)");
        if (rc == FEH_EBREAKDOWN) return set_error(rc, "CG breakdown (some plan)");
        return rc;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_batch_graph_launches(const feh_batch *b) { return b ? b->launches : -1; }


// Inverse of the engineering Voigt strain matrix E[v][l] of nv load cases.
static int voigt_load_inverse(int dim, const double *Ebar_host, std::vector<double> &E) {
    const int nv = dim == 3 ? 6 : 3;
    static const int P2[3][2] = {{0, 0}, {1, 1}, {0, 1}};
    static const int P3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    E.assign(nv * nv, 0.0);
    for (int l = 0; l < nv; ++l)
        for (int v = 0; v < nv; ++v) {
            const int a = dim == 3 ? P3[v][0] : P2[v][0], b = dim == 3 ? P3[v][1] : P2[v][1];
            E[v * nv + l] = Ebar_host[(l * dim + a) * dim + b] * (a == b ? 1.0 : 2.0);
        }
    bool ok = false;
    invert(nv, E, ok);
    if (!ok) return set_error(FEH_EINVAL, "load-case strains are linearly dependent");
    return FEH_OK;
}

int feh_effective_stiffness(int dim, int n_load, const double *Ebar_host, const double *energy_host, double *C_host) {
    if (dim != 2 && dim != 3) return set_error(FEH_EINVAL, "dim must be 2 or 3");
    const int nv = dim == 3 ? 6 : 3;
    if (n_load != nv) return set_error(FEH_EINVAL, "need exactly nv load cases");
    if (!Ebar_host || !energy_host || !C_host) return set_error(FEH_EINVAL, "null argument");
    std::vector<double> E;
    CK(voigt_load_inverse(dim, Ebar_host, E));
    // C = Einv^T W Einv
    std::vector<double> T(nv * nv, 0.0);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s += energy_host[i * nv + k] * E[k * nv + j];
            T[i * nv + j] = s;
        }
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s += E[k * nv + i] * T[k * nv + j];
            C_host[i * nv + j] = s;
        }
    return FEH_OK;
}

int feh_effective_stiffness_weights(int dim, int n_load, const double *Ebar_host, const double *G_host,
                                    double *weight_host) {
    if (dim != 2 && dim != 3) return set_error(FEH_EINVAL, "dim must be 2 or 3");
    const int nv = dim == 3 ? 6 : 3;
    if (n_load != nv) return set_error(FEH_EINVAL, "need exactly nv load cases");
    if (!Ebar_host || !G_host || !weight_host) return set_error(FEH_EINVAL, "null argument");
    std::vector<double> E;  // Einv[l][v]
    CK(voigt_load_inverse(dim, Ebar_host, E));
    // weight = Einv G Einv^T
    std::vector<double> T(nv * nv, 0.0);
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s += E[i * nv + k] * G_host[k * nv + j];
            T[i * nv + j] = s;
        }
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int k = 0; k < nv; ++k) s += T[i * nv + k] * E[j * nv + k];
            weight_host[i * nv + j] = s;
        }
    return FEH_OK;
}

// Mean time of `reps` runs after one warm-up run (events on the plan's stream).
static int time_runs(feh_plan &p, const std::function<int()> &run, int reps, double &ms) {
    hipEvent_t a, b;
    CK(hip_check(hipEventCreate(&a), "event"));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return set_error(FEH_EHIP, "event");
    }
    int rc = run();
    if (rc == FEH_OK) rc = hip_check(hipEventRecord(a, p.stream), "event");
    for (int i = 0; i < reps && rc == FEH_OK; ++i) rc = run();
    if (rc == FEH_OK) rc = hip_check(hipEventRecord(b, p.stream), "event");
    if (rc == FEH_OK) rc = hip_check(hipEventSynchronize(b), "event");
    float t = 0.f;
    if (rc == FEH_OK) rc = hip_check(hipEventElapsedTime(&t, a, b), "event");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    ms = t / reps;
    return rc;
}

int feh_plan_autotune(feh_plan *plan, int reps) {
    try {
        CK(check_plan(plan, false));
        feh_plan &p = *plan;
        if (reps < 1) reps = 3;
        const int D = p.dim;
        // transform zeros: the timing does not depend on the values
        const size_t nvec = (size_t)p.L * D * p.N;
        CK(launch_fill(p, p.ws + p.off_r, nvec, 0.0));
        CK(launch_fill(p, p.ws + p.off_spec, (size_t)p.L * D * p.Nspec * 2, 0.0));
        FftArgs fa;
        fa.r = p.ws + p.off_r;
        fa.spec = p.ws + p.off_spec;
        fa.z = p.ws + p.off_q;
        fa.out_scale = 1.0 / (double)p.N;
        fa.unit_volume = true;  // the CG's scaling: its first-axis pass (compile-time where it has one) is timed
        auto tune_axis = [&](int ax, int len, const std::function<int()> &run, int *geom, int gdef, int gmin) -> int {
            // radix order first (default geometry), then the launch geometry
            double best = 1e30;
            AxisFFT keep = p.fft[ax];
            for (const auto &rad : radix_candidates(len)) {
                AxisFFT cand;
                if (!make_axis(len, rad, cand)) continue;
                p.fft[ax] = cand;
                double ms = 0;
                CK(time_runs(p, run, reps, ms));
                if (ms < best) {
                    best = ms;
                    keep = cand;
                }
            }
            p.fft[ax] = keep;
            if (!geom) return FEH_OK;
            int bestg = 0;
            for (int g = gdef; g >= gmin; g /= 2) {
                *geom = (g == gdef) ? 0 : g;
                double ms = 0;
                CK(time_runs(p, run, reps, ms));
                if (ms < best * 0.98 || g == gdef) {
                    if (g == gdef) best = ms;
                    else { best = ms; bestg = g; }
                }
                if (g == 1) break;
            }
            *geom = bestg;
            return FEH_OK;
        };
        const int PPT = p.prec == FEH_FP32 ? 24 : 16;
        // last axis: forward and inverse
        {
            const int last = D - 1;
            const int nc = p.fft[last].n;
            int rr = std::min((PPT * 256) / (nc * D), 64);
            CK(tune_axis(last, nc, [&]() -> int {
                CK(launch_forward_last(p, fa));
                return launch_inverse_last(p, fa);
            }, &p.tune_rr_last, rr, std::max(1, rr / 4)));
        }
        if (D == 3) {
            int pb = std::min((PPT * 256) / (int)p.n[1], 32);
            CK(tune_axis(1, (int)p.n[1], [&]() -> int {
                CK(launch_middle(p, fa, false));
                return launch_middle(p, fa, true);
            }, &p.tune_pb_mid, pb, std::max(1, pb / 4)));
        }
        {
            const int pb = first_pencils_default(p);
            CK(tune_axis(0, (int)p.n[0], [&]() -> int { return launch_first_fused(p, fa); }, &p.tune_pb_first, pb,
                         std::max(1, pb / 4)));
            // workgroup layout of the axis-0 pass: all load cases per workgroup
            // (inverses cached in registers) or one workgroup per load case
            double best = 1e30;
            int keep = 0;
            for (int v : {-1, 1}) {
                p.tune_first_perlc = v;
                double ms = 0;
                CK(time_runs(p, [&]() -> int { return launch_first_fused(p, fa); }, reps, ms));
                if (ms < best) {
                    best = ms;
                    keep = v;
                }
            }
            p.tune_first_perlc = keep;
        }
        if (D == 3) {
            // stencil tile rows (8 or 16 rows of 32 voxels)
            StencilArgs sa;
            sa.in0 = p.ws + p.off_r;
            sa.out0 = p.ws + p.off_q;
            double best = 1e30;
            int keep = 8;
            for (int vy : {8, 16}) {
                p.tune_stencil_vy = vy;
                double ms = 0;
                CK(time_runs(p, [&]() -> int { return launch_stencil(p, ST_APPLY, sa); }, reps, ms));
                if (ms < best) {
                    best = ms;
                    keep = vy;
                }
            }
            p.tune_stencil_vy = keep;
        }
        return hip_check(hipStreamSynchronize(p.stream), "autotune");
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_plan_set_tuning(feh_plan *plan, const int *values, int n_values) {
    try {
        if (!plan || !values) return set_error(FEH_EINVAL, "null argument");
        feh_plan &p = *plan;
        if (n_values < 5) return set_error(FEH_EINVAL, "schedule too short");
        const int rr = values[0], pbm = values[1], pbf = values[2], perlc = values[3], rows = values[4];
        if (rr < 0 || pbm < 0 || pbf < 0) return set_error(FEH_EINVAL, "workgroup sizes must be >= 0");
        if (pbf > 0 && pbf < std::max(1, first_pencils_default(p) / 4))
            return set_error(FEH_EINVAL, "axis-0 pencils per workgroup below a quarter of the default");
        if (perlc != 0 && perlc != 1) return set_error(FEH_EINVAL, "axis-0 layout must be 0 or 1");
        if (p.dim == 3 ? (rows != 8 && rows != 16) : rows != 1)
            return set_error(FEH_EINVAL, "stencil rows must be 8 or 16 (3D) or 1 (2D)");
        AxisFFT ax[3] = {p.fft[0], p.fft[1], p.fft[2]};
        int i = 5;
        for (int a = 0; a < 3; ++a) {
            if (i >= n_values) return set_error(FEH_EINVAL, "schedule too short");
            const int np = values[i++];
            if (np < 0 || i + np > n_values) return set_error(FEH_EINVAL, "schedule too short");
            std::vector<int> rad(values + i, values + i + np);
            i += np;
            if (a >= p.dim) {
                if (np != 0) return set_error(FEH_EINVAL, "passes given for a missing axis");
                continue;
            }
            const int len = p.fft[a].n;
            for (int r : rad) {
                // butterfly radices, or a prime above 13 (direct-DFT pass)
                bool ok = r == 2 || r == 3 || r == 4 || r == 5 || r == 7 || r == 8 || r == 11 || r == 13;
                if (!ok && r > 13) {
                    ok = true;
                    for (int f = 2; f * f <= r; ++f)
                        if (r % f == 0) ok = false;
                }
                if (!ok) return set_error(FEH_EINVAL, "radices must be 2, 3, 4, 5, 7, 8, 11, 13 or a prime above 13");
            }
            if (!make_axis(len, rad, ax[a])) return set_error(FEH_EINVAL, "radices do not multiply to the axis length");
        }
        // optional trailing value: compile-time transforms allowed (1) or not (0)
        int ct = p.tune_ct;
        if (i < n_values) {
            ct = values[i++];
            if (ct != 0 && ct != 1) return set_error(FEH_EINVAL, "compile-time transform flag must be 0 or 1");
        }
        for (int a = 0; a < 3; ++a) p.fft[a] = ax[a];
        p.tune_ct = ct;
        p.tune_rr_last = rr;
        p.tune_pb_mid = pbm;
        p.tune_pb_first = pbf;
        p.tune_first_perlc = perlc ? 1 : -1;
        p.tune_stencil_vy = p.dim == 3 ? rows : 0;
        return FEH_OK;
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_plan_cg_residual_spectral(const feh_plan *plan) {
    if (!plan) return set_error(FEH_EINVAL, "null plan");
    return cg_residual_spectral(*plan) ? 1 : 0;
}

int feh_plan_tuning(const feh_plan *plan, int *values, int n_values) {
    if (!plan || !values) return set_error(FEH_EINVAL, "null argument");
    std::vector<int> v = {plan->tune_rr_last, plan->tune_pb_mid, plan->tune_pb_first,
                          first_per_load_case(*plan) ? 1 : 0, stencil_rows(*plan)};
    for (int a = 0; a < 3; ++a) {
        const int np = a < plan->dim ? plan->fft[a].npass : 0;
        v.push_back(np);
        for (int s = 0; s < np; ++s) v.push_back(plan->fft[a].pass[s].R);
    }
    v.push_back(plan->tune_ct);
    for (int i = 0; i < n_values; ++i) values[i] = i < (int)v.size() ? v[i] : 0;
    return (int)v.size();
}

int feh_profile_enable(feh_plan *plan, int enable) {
    if (!plan) return set_error(FEH_EINVAL, "null plan");
    plan->prof_on = enable != 0;
    plan->prof_used = 0;
    for (int k = 0; k < feh_plan::kProfKinds; ++k) {
        plan->prof_ms[k] = 0.0;
        plan->prof_n[k] = 0;
    }
    return FEH_OK;
}

int feh_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, void *hip_stream) {
    if (!dst_dev || !src_dev) return set_error(FEH_EINVAL, "null argument");
    if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst_dev) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(src_dev) % 16 != 0)
        return set_error(FEH_EINVAL, "stream copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    const char *d = static_cast<const char *>(dst_dev), *s = static_cast<const char *>(src_dev);
    if (d < s + bytes && s < d + bytes) return set_error(FEH_EINVAL, "stream copy buffers overlap");
    if (bytes == 0) return FEH_OK;
    return launch_stream_copy(dst_dev, src_dev, bytes / 16, static_cast<hipStream_t>(hip_stream));
}

int feh_profile_read(const feh_plan *plan, double *ms_total, int64_t *launches, int n_kinds) {
    if (!plan || !ms_total || !launches) return set_error(FEH_EINVAL, "null argument");
    for (int k = 0; k < n_kinds; ++k) {
        ms_total[k] = k < feh_plan::kProfKinds ? plan->prof_ms[k] : 0.0;
        launches[k] = k < feh_plan::kProfKinds ? plan->prof_n[k] : 0;
    }
    return FEH_OK;
}

// Sensitivity pass shared by feh_energy_sensitivity (grad_E_dev null: the
// two Lame fields) and feh_energy_sensitivity_E (grad_lam_dev, grad_mu_dev
// null: the Young's modulus field through the plane-strain Lame maps at the
// nu the material was set with).
static int sensitivity(feh_plan *plan, const double *weight_host, void *grad_lam_dev, void *grad_mu_dev,
                       void *grad_E_dev) {
    try {
        CK(check_plan(plan, true));
        feh_plan &p = *plan;
        if (!weight_host || (!grad_E_dev && (!grad_lam_dev || !grad_mu_dev))) return set_error(FEH_EINVAL, "null argument");
        double aE = 0.0, bE = 0.0;
        if (grad_E_dev) {
            if (!(p.field_nu > -1.0 && p.field_nu < 0.5))
                return set_error(FEH_EINVAL, "the material was not set by feh_set_material_field");
            const double nu = p.field_nu;
            aE = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));  // d lambda / d E
            bE = 1.0 / (2.0 * (1.0 + nu));             // d mu / d E
        }
        if (!p.solved) return set_error(FEH_EINVAL, "no solution in the plan (call feh_solve first)");
        for (int i = 0; i < p.L * p.L; ++i)
            if (!std::isfinite(weight_host[i])) return set_error(FEH_EINVAL, "weights must be finite");
        for (int l = 0; l < p.L; ++l)
            for (int m = 0; m < p.L; ++m)
                if (l / p.G != m / p.G && weight_host[l * p.L + m] != 0.0)
                    return set_error(FEH_EINVAL, "weights across microstructures must be zero");
        std::vector<int> pl, pm, gofs(1, 0);
        std::vector<double> pw;
        for (int b = 0; b < p.nbatch; ++b) {
            for (int l = b * p.G; l < (b + 1) * p.G; ++l)
                for (int m = l; m < (b + 1) * p.G; ++m) {
                    const double w = (l == m) ? weight_host[l * p.L + l] : weight_host[l * p.L + m] + weight_host[m * p.L + l];
                    if (w == 0.0) continue;
                    pl.push_back(l);
                    pm.push_back(m);
                    pw.push_back(w);
                }
            gofs.push_back((int)pl.size());
        }
        const int np = (int)pl.size();
        const size_t ni = (size_t)kMaxLoad * (kMaxLoad + 1) / 2;
        int *dpl = p.ptr<int>(p.off_pairs);
        int *dpm = dpl + ni;
        int *dgo = dpm + ni;  // kMaxLoad + 1 entries
        double *dpw = reinterpret_cast<double *>(dgo + 2 * kMaxLoad);
        if (np > 0) {
            CK(hip_check(hipMemcpyAsync(dpl, pl.data(), np * sizeof(int), hipMemcpyHostToDevice, p.stream), "pairs"));
            CK(hip_check(hipMemcpyAsync(dpm, pm.data(), np * sizeof(int), hipMemcpyHostToDevice, p.stream), "pairs"));
            CK(hip_check(hipMemcpyAsync(dpw, pw.data(), np * sizeof(double), hipMemcpyHostToDevice, p.stream), "pairs"));
        }
        CK(hip_check(hipMemcpyAsync(dgo, gofs.data(), gofs.size() * sizeof(int), hipMemcpyHostToDevice, p.stream), "pairs"));
        bool offdiag = false;
        for (int q = 0; q < np; ++q) offdiag = offdiag || pl[q] != pm[q];
        CK(launch_sensitivity(p, p.ws + p.off_u, p.ptr<double>(p.off_ebar), dpl, dpm, dpw, dgo, offdiag, grad_lam_dev,
                              grad_mu_dev, grad_E_dev, aE, bE));
        return hip_check(hipStreamSynchronize(p.stream), "sensitivity");
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_energy_sensitivity(feh_plan *plan, const double *weight_host, void *grad_lam_dev, void *grad_mu_dev) {
    if (!grad_lam_dev || !grad_mu_dev) return set_error(FEH_EINVAL, "null argument");
    return sensitivity(plan, weight_host, grad_lam_dev, grad_mu_dev, nullptr);
}

int feh_energy_sensitivity_E(feh_plan *plan, const double *weight_host, void *grad_E_dev) {
    if (!grad_E_dev) return set_error(FEH_EINVAL, "null argument");
    return sensitivity(plan, weight_host, nullptr, nullptr, grad_E_dev);
}

int feh_apply_operator(feh_plan *plan, const void *p_dev, void *q_dev) {
    CK(check_plan(plan, true));
    if (!p_dev || !q_dev) return set_error(FEH_EINVAL, "null argument");
    feh_plan &p = *plan;
    CK(launch_aos_to_soa(p, p_dev, p.ws + p.off_p));
    StencilArgs sa;
    sa.in0 = p.ws + p.off_p;
    sa.out0 = p.ws + p.off_q;
    CK(launch_stencil(p, ST_APPLY, sa));
    CK(launch_soa_to_aos(p, p.ws + p.off_q, q_dev));
    return hip_check(hipStreamSynchronize(p.stream), "apply operator");
}

int feh_apply_preconditioner(feh_plan *plan, const void *r_dev, void *z_dev) {
    CK(check_plan(plan, false));
    if (!r_dev || !z_dev) return set_error(FEH_EINVAL, "null argument");
    feh_plan &p = *plan;
    CK(launch_aos_to_soa(p, r_dev, p.ws + p.off_r));
    CK(precondition(p, p.ws + p.off_r, p.ws + p.off_q, nullptr, nullptr, false));
    CK(launch_soa_to_aos(p, p.ws + p.off_q, z_dev));
    return hip_check(hipStreamSynchronize(p.stream), "apply preconditioner");
}

int feh_apply_projection(feh_plan *plan, const void *e_dev, void *Ge_dev) {
    CK(check_plan(plan, false));
    if (!e_dev || !Ge_dev) return set_error(FEH_EINVAL, "null argument");
    feh_plan &p = *plan;
    StencilArgs sa;
    sa.in0 = e_dev;
    sa.out0 = p.ws + p.off_q;
    sa.identity_material = true;
    CK(launch_stencil(p, ST_DIV, sa));
    CK(precondition(p, p.ws + p.off_q, p.ws + p.off_q, nullptr, nullptr, false));
    CK(launch_grad(p, p.ws + p.off_q, Ge_dev));
    return hip_check(hipStreamSynchronize(p.stream), "apply projection");
}

int feh_fft_forward(feh_plan *plan, const void *x_dev, void *X_dev) {
    CK(check_plan(plan, false));
    if (!x_dev || !X_dev) return set_error(FEH_EINVAL, "null argument");
    feh_plan &p = *plan;
    FftArgs fa;
    fa.r = x_dev;
    fa.spec = p.ws + p.off_spec;
    CK(launch_forward_last(p, fa));
    if (p.dim == 3) CK(launch_middle(p, fa, false));
    CK(launch_first(p, fa, false));
    CK(launch_spec_to_numpy(p, p.ws + p.off_spec, X_dev, true));
    return hip_check(hipStreamSynchronize(p.stream), "fft forward");
}

// ---------------------------------------------------------------------------
// allocation-free solve: the workspace is a file-scope device array
// ---------------------------------------------------------------------------
int feh_solve_noalloc(feh_plan *plan, const void *lambda_dev, const void *mu_dev, const double *Ebar_host,
                      double tol, int max_iter, const void *u0_dev, void *u_dev, void *strain_dev, void *stress_dev,
                      double *stress_mean_host, double *energy_host, feh_report *report_host) {
    try {
        const double t0 = wall_seconds();
        if (!plan) return set_error(FEH_EINVAL, "null plan");
        if (!lambda_dev || !mu_dev) return set_error(FEH_EINVAL, "null material pointer");
        feh_plan &p = *plan;
        if (p.prof_on) return set_error(FEH_EINVAL, "profiling creates events; disable it for feh_solve_noalloc");
        if (p.total > kStaticScratchBytes)
            return set_error(FEH_ENOMEM, "the plan needs " + std::to_string(p.total) +
                                             " bytes of workspace, more than the static scratch of " +
                                             std::to_string(kStaticScratchBytes) + " bytes");
        char *ws = nullptr;
        CK(static_scratch(p.stream, &ws));
        // borrow the static array as the workspace; the plan's own workspace,
        // material and last solution are left as they were
        char *const own_ws = p.ws;
        const size_t own_bytes = p.ws_bytes;
        const bool own_material = p.material_set, own_solved = p.solved;
        const double own_nu = p.field_nu;
        p.ws = ws;
        p.ws_bytes = kStaticScratchBytes;
        int rc = upload_tables(p);
        if (rc == FEH_OK) {
            int *flag = p.ptr<int>(p.off_flag);
            rc = launch_fill(p, flag, 1, 0.0);
            if (rc == FEH_OK) rc = launch_material_lame(p, lambda_dev, mu_dev, flag);
            if (rc == FEH_OK) rc = read_flag(p, flag, "feh_solve_noalloc");
        }
        if (rc == FEH_OK) {
            p.material_set = true;
            rc = solve_all(p, Ebar_host, tol, max_iter, u0_dev, u_dev, strain_dev, stress_dev, stress_mean_host,
                           energy_host, report_host);
            if (rc == FEH_OK || rc == FEH_ENOCONV || rc == FEH_EBREAKDOWN) stamp_reports(report_host, p.L, t0);
        }
        p.ws = own_ws;
        p.ws_bytes = own_bytes;
        p.material_set = own_material;
        p.solved = own_solved;
        p.field_nu = own_nu;
        return rc;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

int feh_fft_inverse(feh_plan *plan, const void *X_dev, void *x_dev) {
    CK(check_plan(plan, false));
    if (!x_dev || !X_dev) return set_error(FEH_EINVAL, "null argument");
    feh_plan &p = *plan;
    FftArgs fa;
    fa.spec = p.ws + p.off_spec;
    fa.z = x_dev;
    fa.out_scale = 1.0 / (double)p.N;
    CK(launch_spec_to_numpy(p, X_dev, p.ws + p.off_spec, false));
    CK(launch_first(p, fa, true));
    if (p.dim == 3) CK(launch_middle(p, fa, true));
    CK(launch_inverse_last(p, fa));
    return hip_check(hipStreamSynchronize(p.stream), "fft inverse");
}

}  // extern "C"
