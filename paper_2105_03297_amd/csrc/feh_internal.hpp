// Internal declarations of the FE-projection homogenization library.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "feh.h"

namespace feh {

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------------------
// limits and shapes
// ---------------------------------------------------------------------------
constexpr int kMaxRadixCount = 16;
constexpr int kMaxLoad = 64;
constexpr int kMaxN = 4096;
constexpr int kMaxPhase = 4096;

// Division by a runtime constant d < 2^31 for dividends x < 2^31:
// q = (umulhi(x, mul) + x) >> sh  (round-up multiplier method).
struct FastDiv {
    uint32_t d = 1, mul = 1, sh = 0;
    static FastDiv make(uint32_t d) {
        FastDiv f;
        f.d = d;
        uint32_t l = 0;
        while ((1ull << l) < d) ++l;
        f.sh = l;
        f.mul = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
        return f;
    }
#ifdef __HIP_DEVICE_COMPILE__
    __device__ __forceinline__ uint32_t div(uint32_t x) const { return (__umulhi(x, mul) + x) >> sh; }
#else
    uint32_t div(uint32_t x) const { return (uint32_t)((((uint64_t)x * mul) >> 32) + x) >> sh; }
#endif
};

struct PassInfo {
    int R = 1;        // radix
    int Lstar = 1;    // product of the radices of the earlier passes
    FastDiv m;        // n / (Lstar * R)
};

struct AxisFFT {
    int n = 1;        // transform length (n/2 for the packed last axis)
    int npass = 0;
    PassInfo pass[kMaxRadixCount];
};

// Per-load-case CG state, kept on the device (FP64).
struct LcState {
    double rho;        // r.z of the current iterate
    double rho_ref;    // f.M^+f (reference for the relative residual)
    double pq;         // p.q of the current iteration
    double alpha;      // rho / pq
    double beta;       // rho_new / rho
    double alpha_pend; // u += alpha_pend * p still to be applied
    double relres;     // sqrt(rho / rho_ref)
    int active;        // 1 while iterating
    int iters;         // completed iterations
    int status;        // FEH_OK / FEH_ENOCONV / FEH_EBREAKDOWN
    int pad;
};

// Solve parameters read by the scalar kernels.
struct SolveParams {
    double tol;
    int max_iter;
    int n_load;
};

}  // namespace feh

// ---------------------------------------------------------------------------
// the plan
// ---------------------------------------------------------------------------
struct feh_plan {
    int dim = 0;
    int64_t n[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    int L = 1;            // load cases in the plan: nbatch groups of G
    int nbatch = 1;       // microstructures of this shape (one material each)
    int G = 1;            // load cases per microstructure; load case l uses material l / G
    int prec = FEH_FP64;
    hipStream_t stream = nullptr;

    int64_t N = 0;        // voxels (= nodes)
    int64_t nh = 0;       // last-axis half-spectrum length n_last/2 + 1
    int64_t Nspec = 0;    // complex points per component: N / n_last * nh
    int ne = 0;           // elements per voxel
    size_t rsize = 8;     // bytes per real

    feh::AxisFFT fft[3];  // per axis (last axis: packed length n/2 when even)
    bool last_even = true;

    // workspace layout (byte offsets)
    size_t off_u = 0, off_r = 0, off_p = 0, off_q = 0;
    size_t off_spec = 0, off_lam = 0, off_mu = 0;
    size_t off_tw[3] = {0, 0, 0};       // twiddles e^{-2 pi i j / n_a}, j < n_a (plan precision)
    size_t off_om[3] = {0, 0, 0};       // e^{+2 pi i m / n_a} (FP64)
    size_t off_aa[3] = {0, 0, 0};       // (e^{+2 pi i m / n_a} - 1) / h_a (FP64)
    size_t off_tab = 0, off_ebar = 0, off_sums = 0;
    size_t off_part = 0, off_state = 0, off_flag = 0;
    size_t off_pairs = 0;               // load-case pair list of the sensitivity pass
    size_t off_minv = 0;                // per-wavevector (B^*B)^-1 table of the CG's first-axis pass
    size_t part_stride = 0;             // doubles per load case in the partials
    size_t total = 0;

    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool material_set = false;
    double field_nu = -2.0;             // nu of feh_set_material_field (outside (-1, 0.5): other setter)
    // launch geometry chosen by feh_plan_autotune (0: the default heuristic);
    // the radix orders are the pass lists of fft[]
    int tune_rr_last = 0;               // rows per workgroup, last axis
    int tune_pb_mid = 0;                // pencils per workgroup, axis 1 (3D)
    int tune_pb_first = 0;              // pencils per workgroup, axis 0
    int tune_stencil_vy = 0;            // 3D stencil tile rows (8 or 16; 0: default)
    int tune_first_perlc = 0;           // axis-0 pass: 1 one workgroup per load case, -1 all load cases, 0 default
    int tune_ct = 1;                    // 1: compile-time transforms where the shape has one, 0: run-time passes only
    bool solved = false;                // off_u holds the fluctuations of the last feh_solve
    // the (B^*B)^-1 table at off_minv: built for this workspace and pencil
    // block size (0: not built); rebuilt by the first-axis launcher on change
    mutable const char *minv_ws = nullptr;
    mutable int minv_pb = 0;
    mutable int minv_q = -1;            // slot interleave of the table (0: plain order)

    // optional per-kernel event timing of the CG loop
    static constexpr int kProfKinds = 8;
    bool prof_on = false;
    mutable std::vector<hipEvent_t> prof_ev;  // pool: (start, end) pairs
    mutable std::vector<int> prof_kind;       // kind of each recorded pair
    mutable size_t prof_used = 0;             // pairs recorded since the last drain
    mutable double prof_ms[kProfKinds] = {0};
    mutable long long prof_n[kProfKinds] = {0};
    mutable long long prof_lc_launches[kProfKinds] = {0};  // load-case launches (active ones)

    // host copies of the tables (uploaded by set_workspace)
    std::vector<double> tw_host[3];     // interleaved re, im in FP64
    std::vector<double> om_host[3], aa_host[3];

    template <typename P>
    P *ptr(size_t off) const { return reinterpret_cast<P *>(ws + off); }
};

namespace feh {

// error helpers (capi.hip)
int set_error(int code, const std::string &msg);
int hip_check(hipError_t e, const char *what);

// Host wall clock (seconds) and the stamp of a call's duration into its
// reports (every load case of one call gets the same value).
inline double wall_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
inline void stamp_reports(feh_report *rep, int n, double t0) {
    if (!rep) return;
    const double dt = wall_seconds() - t0;
    for (int i = 0; i < n; ++i) rep[i].seconds = dt;
}

// return the error code of a failing call
#define CK(...)                          \
    do {                                 \
        int rc__ = (__VA_ARGS__);        \
        if (rc__ != FEH_OK) return rc__; \
    } while (0)

// ---------------------------------------------------------------------------
// kernel launchers (defined in the kern_*.hip files)
// ---------------------------------------------------------------------------
// Stencil modes.
enum StencilMode {
    ST_APPLY = 0,   // q = K p
    ST_CG = 1,      // p_new = z + beta p_old (or z), q = K p_new, u += alpha_pend p_old, partial p.q
    ST_RESID = 2,   // r = -B^T C (Ebar + B u)   (u may be null: right-hand side)
    ST_DIV = 3      // q = B^T C e for the element field e (projection test export)
};

struct StencilArgs {
    const void *in0 = nullptr;   // p (APPLY, CG), u (RESID, nullable)
    void *out0 = nullptr;        // q (APPLY, CG), r (RESID)
    const double *Ebar = nullptr;// device [L][D][D] (RESID)
    double *partial = nullptr;   // [L][part_stride] (CG)
    const LcState *state = nullptr;
    bool identity_material = false;  // lambda = 0, mu = 1/2 (preconditioner tests)
    // element volume divided by the voxel volume (1/6, 1/2) instead of the
    // true volume: the CG paths scale K, f and M by the same constant, which
    // leaves every iterate unchanged and keeps FP32 stencils in range at any
    // voxel size; the test exports use the true volume
    bool unit_volume = false;
};

int launch_stencil(const feh_plan &p, int mode, const StencilArgs &a);

// FFT pipeline pieces (kern_fft.hip)
struct FftArgs {
    const void *r = nullptr;     // real input (SoA [L][D][N])
    const void *q = nullptr;     // fused axpy: r -= alpha q (nullable)
    void *r_out = nullptr;       // updated r (fused axpy)
    void *spec = nullptr;        // half spectrum [L][n0][..][nh][D]
    const void *spec_in = nullptr;  // forward middle (3D) / first-axis (2D) pass: read here, write spec (null: in place)
    bool rspec = false;          // forward last pass: spec (the residual's last-axis half spectrum) -= alpha q^
    void *z = nullptr;           // real output
    void *p_upd = nullptr;       // CG update fused into the last inverse pass (nullable):
    void *u_upd = nullptr;       //   u += alpha_pend p, then p = z + beta p, in place (z not stored)
    double *partial = nullptr;   // Parseval r.z partials
    const LcState *state = nullptr;  // active mask, alpha (nullable: all active, no axpy)
    double out_scale = 1.0;      // c2r output scale
    int ksolve = 1;              // apply (B^*B)^-1 between forward and inverse first axis
    bool identity_test = false;  // forward/inverse only (no k-solve)
    int comps = 0;               // components per point (0: the dimension)
    bool unit_volume = false;    // M formed with the element volume over the voxel volume (CG paths)
};

int launch_forward_last(const feh_plan &p, const FftArgs &a);   // r2c along the last axis
int launch_middle(const feh_plan &p, const FftArgs &a, bool inverse);  // c2c axis 1 (3D)
int launch_first_fused(const feh_plan &p, const FftArgs &a);    // c2c axis 0 fwd, k-solve, inv
int launch_first(const feh_plan &p, const FftArgs &a, bool inverse);  // c2c axis 0 only
int launch_first_plain(const feh_plan &p, const FftArgs &a, bool inverse);  // c2c axis 0, any a.comps
int launch_inverse_last(const feh_plan &p, const FftArgs &a);   // c2r along the last axis
bool last_ct_ok(const feh_plan &p, int D);      // the last-axis passes take the compile-time transform
// the CG keeps its residual as a last-axis half spectrum (FP32, compile-time last-axis passes)
bool cg_residual_spectral(const feh_plan &p);

// scalar / vector kernels (kern_cg.hip)
int launch_fill(const feh_plan &p, void *x, size_t count, double value);
int launch_stream_copy(void *dst, const void *src, size_t n16, hipStream_t stream);
int launch_aos_to_soa(const feh_plan &p, const void *aos, void *soa);
int launch_soa_to_aos(const feh_plan &p, const void *soa, void *aos);
int launch_init_state(const feh_plan &p, LcState *st, int n_load);
int launch_finish_rho(const feh_plan &p, LcState *st, const double *partial, int nparts, int mode,
                      double tol, int max_iter);
int launch_finish_pq(const feh_plan &p, LcState *st, const double *partial, int nparts);
// the same with an explicit partial-sum stride (doubles per load case)
int launch_finish_rho_stride(const feh_plan &p, LcState *st, const double *partial, int nparts, int stride,
                             int mode, double tol, int max_iter);
int launch_finish_pq_stride(const feh_plan &p, LcState *st, const double *partial, int nparts, int stride);
int launch_finalize_u(const feh_plan &p, void *u, const void *pv, const LcState *st);
int launch_material_lame(const feh_plan &p, const void *lam, const void *mu, int *flag);
int launch_material_phases(const feh_plan &p, const int32_t *phase, const double *tab, int n_phase,
                           int *flag);
int launch_material_field(const feh_plan &p, const void *E, double nu, int *flag);
int launch_spec_to_numpy(const feh_plan &p, const void *spec, void *out, bool to_numpy);
// subtract the per-(load case, component) mean of an SoA nodal field
int launch_remove_mean(const feh_plan &p, void *x, double *partial, double *mean);

// post-processing and projection helpers (kern_post.hip)
// sums[l*ns + k] = <sigma>_l (symmetric components), sums[L*ns + pair(l<=m)] = W_lm
int launch_post_sums(const feh_plan &p, const void *u, const double *Ebar_dev, void *strain, void *stress,
                     double *partial, double *sums);
int launch_grad(const feh_plan &p, const void *u, void *e);   // e = sym(B u) element field
// g_lam, g_mu [nbatch][N] = sum over the pairs of each microstructure (l <= m,
// weight w; pairs gofs[b] .. gofs[b+1] - 1) of the voxel's share of dW_lm/dlambda, dW_lm/dmu
// g_E non-null: write g_E = aE g_lam + bE g_mu instead of the two fields;
// offdiag: some pair has l != m
int launch_sensitivity(const feh_plan &p, const void *u, const double *Ebar_dev, const int *pl, const int *pm,
                       const double *pw, const int *gofs, bool offdiag, void *g_lam, void *g_mu, void *g_E,
                       double aE, double bE);
int post_num_slots(const feh_plan &p);

// partial-sum sizes
int stencil_num_parts(const feh_plan &p);
int stencil_rows(const feh_plan &p);           // 3D stencil tile rows in use
int first_num_parts(const feh_plan &p);
int first_pencils_default(const feh_plan &p);  // before tuning
int first_ct_pencils(const feh_plan &p);       // compile-time CG pass block size (0: none)
bool first_per_load_case(const feh_plan &p);   // axis-0 pass layout (workgroup per load case)
int post_num_parts(const feh_plan &p);

}  // namespace feh
