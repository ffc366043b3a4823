// CG scalar updates, vector utilities and material set-up.
//
// The CG scalars of every load case live on the device (LcState, FP64), so a
// chunk of iterations runs without host round trips; the host polls the
// active flags between chunks.  Reductions over per-block partial sums use a
// fixed summation order, so repeated solves are bitwise identical.
#include <algorithm>

#include "device_common.hpp"

namespace feh {
namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ void k_fill(T *x, long long n, T v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

// [L][N][D] <-> [L][D][N]
template <typename T, bool TO_SOA>
__global__ void k_transpose(const T *in, T *out, long long N, int D, int L) {
    const long long total = N * D * L;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        // i indexes the output
        if (TO_SOA) {
            const long long n = i % N;
            const long long lc_c = i / N;
            const int c = (int)(lc_c % D);
            const long long lc = lc_c / D;
            out[i] = in[(lc * N + n) * D + c];
        } else {
            const int c = (int)(i % D);
            const long long lc_n = i / D;
            const long long n = lc_n % N;
            const long long lc = lc_n / N;
            out[i] = in[(lc * D + c) * N + n];
        }
    }
}

__global__ void k_init_state(LcState *st, int L) {
    const int l = threadIdx.x;
    if (l < L) {
        LcState s{};
        s.active = 1;
        st[l] = s;
    }
}

__device__ double sum_parts(const double *part, int n, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) v += part[i];
    return block_sum<kThreads>(v, sh);
}

// mode 0: reference norm f.M^+f; mode 1: initial r.z (also the reference when
// ref_too); mode 2: iteration update (rho_new, convergence, beta).
__global__ void k_finish_rho(LcState *st, const double *part, int nparts, int stride, int mode, int ref_too,
                             double tol, int max_iter) {
    __shared__ double sh[kThreads / 64];
    const int l = blockIdx.x;
    LcState &s = st[l];
    if (mode == 2 && !s.active) return;
    const double v = sum_parts(part + (long long)l * stride, nparts, sh);
    if (threadIdx.x != 0) return;
    if (mode == 0) {
        s.rho_ref = v;
        return;
    }
    if (mode == 1) {
        // reference f.M^+f; a warm start with f = 0 measures against its own
        // initial residual instead
        if (ref_too || !(s.rho_ref > 0.0)) s.rho_ref = v;
        s.rho = v;
        const double ref = s.rho_ref;
        if (!isfinite(v) || !isfinite(ref)) {
            s.active = 0;
            s.status = FEH_EBREAKDOWN;
            return;
        }
        if (!(v > 0.0)) {
            // zero residual (e.g. homogeneous material): nothing to iterate
            s.relres = 0.0;
            s.active = 0;
            return;
        }
        s.relres = sqrt(v / ref);
        if (s.relres <= tol) s.active = 0;
        return;
    }
    // mode 2
    s.iters += 1;
    if (!isfinite(v)) {
        s.active = 0;
        s.status = FEH_EBREAKDOWN;
        return;
    }
    const double rr = v > 0.0 ? v : 0.0;
    s.relres = sqrt(rr / s.rho_ref);
    if (s.relres <= tol) {
        s.active = 0;
        s.status = FEH_OK;
        return;
    }
    if (s.iters >= max_iter) {
        s.active = 0;
        s.status = FEH_ENOCONV;
        return;
    }
    s.beta = rr / s.rho;
    s.rho = rr;
}

__global__ void k_finish_pq(LcState *st, const double *part, int nparts, int stride) {
    __shared__ double sh[kThreads / 64];
    const int l = blockIdx.x;
    LcState &s = st[l];
    if (!s.active) return;
    const double v = sum_parts(part + (long long)l * stride, nparts, sh);
    if (threadIdx.x != 0) return;
    s.pq = v;
    if (!(v > 0.0) || !isfinite(v)) {
        s.active = 0;
        s.status = FEH_EBREAKDOWN;
        s.alpha = 0.0;
        s.alpha_pend = 0.0;
        return;
    }
    s.alpha = s.rho / v;
    s.alpha_pend = s.alpha;
}

// u += alpha_pend * p for every load case (the update still pending when a
// load case stopped), then clear the pending step.
template <typename T>
__global__ void k_finalize_u(T *u, const T *p, const LcState *st, long long per_lc, int L) {
    const long long total = per_lc * L;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int l = (int)(i / per_lc);
        const double a = st[l].alpha_pend;
        if (a != 0.0) u[i] += T(a) * p[i];
    }
}

__global__ void k_clear_pending(LcState *st, int L) {
    if ((int)threadIdx.x < L) st[threadIdx.x].alpha_pend = 0.0;
}

template <typename T>
__global__ void k_mat_lame(const T *lam, const T *mu, T *ol, T *om, long long N, int dim, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const T l = lam[i], m = mu[i];
        if (!isfinite(l) || !isfinite(m) || m < T(0) || l + T(2) * m / T(dim) < T(0)) atomicOr(flag, 1);
        ol[i] = l;
        om[i] = m;
    }
}

__global__ void k_mat_phases_d(const int *ph, const double *tab, int nph, double *ol, double *om, long long N, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const int k = ph[i];
        if (k < 0 || k >= nph) {
            atomicOr(flag, 1);
            ol[i] = 0.0;
            om[i] = 0.0;
        } else {
            ol[i] = tab[2 * k];
            om[i] = tab[2 * k + 1];
        }
    }
}

__global__ void k_mat_phases_f(const int *ph, const double *tab, int nph, float *ol, float *om, long long N, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const int k = ph[i];
        if (k < 0 || k >= nph) {
            atomicOr(flag, 1);
            ol[i] = 0.f;
            om[i] = 0.f;
        } else {
            ol[i] = (float)tab[2 * k];
            om[i] = (float)tab[2 * k + 1];
        }
    }
}

template <typename T>
__global__ void k_mat_field(const T *E, T *ol, T *om, long long N, double cl, double cm, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
        const T e = E[i];
        if (!isfinite(e) || e < T(0)) atomicOr(flag, 1);
        ol[i] = T(cl * double(e));
        om[i] = T(cm * double(e));
    }
}

// internal spectrum [L][n0][..][nh][D] <-> numpy rfftn layout [L*D][n0][..][nh]
template <typename T>
__global__ void k_spec_numpy(const Cx<T> *in, Cx<T> *out, long long Nspec, int D, int L, int to_numpy) {
    const long long total = Nspec * D * L;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        // i indexes the numpy layout: (lc*D + c) * Nspec + s
        const long long s = i % Nspec;
        const long long lcc = i / Nspec;
        const int c = (int)(lcc % D);
        const long long lc = lcc / D;
        const long long j = (lc * Nspec + s) * D + c;
        if (to_numpy) out[i] = in[j];
        else out[j] = in[i];
    }
}

// mean removal of an SoA field [L*D][N]: per-block partial sums, a fixed-order
// finish, then subtraction
__global__ void k_mean_partial_d(const double *x, long long N, int nblk, double *part) {
    __shared__ double red[kThreads / 64];
    const int f = blockIdx.y;
    double v = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < N; i += (long long)nblk * kThreads)
        v += x[(long long)f * N + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) part[(long long)f * nblk + blockIdx.x] = s;
}
__global__ void k_mean_partial_f(const float *x, long long N, int nblk, double *part) {
    __shared__ double red[kThreads / 64];
    const int f = blockIdx.y;
    double v = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < N; i += (long long)nblk * kThreads)
        v += (double)x[(long long)f * N + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) part[(long long)f * nblk + blockIdx.x] = s;
}
__global__ void k_mean_finish(const double *part, int nblk, double *mean, double invN) {
    __shared__ double red[kThreads / 64];
    const int f = blockIdx.x;
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) v += part[(long long)f * nblk + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) mean[f] = s * invN;
}
template <typename T>
__global__ void k_sub_mean(T *x, long long N, int nf, const double *mean) {
    const long long total = N * nf;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x)
        x[i] -= T(mean[i / N]);
}

int grid_for(long long n) {
    long long g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// Streaming copy of n 16-byte words with nontemporal loads and stores: the
// attainable read+write bandwidth of the device, measured beside the kernels.
__global__ __launch_bounds__(kThreads) void k_stream_copy(const void *__restrict__ src, void *__restrict__ dst,
                                                          long long n) {
    typedef unsigned int U4 __attribute__((ext_vector_type(4)));
    const U4 *a = static_cast<const U4 *>(src);
    U4 *b = static_cast<U4 *>(dst);
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

}  // namespace

int launch_stream_copy(void *dst, const void *src, size_t n16, hipStream_t stream) {
    const long long n = (long long)n16;
    const long long want = (n + kThreads - 1) / kThreads;
    const int g = (int)std::max(1LL, std::min(want, 32768LL));
    hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(kThreads), 0, stream, src, dst, n);
    return hip_check(hipGetLastError(), "stream copy launch");
}

int launch_fill(const feh_plan &p, void *x, size_t count, double value) {
    const int g = grid_for((long long)count);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(kThreads), 0, p.stream, (double *)x, (long long)count, value);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(kThreads), 0, p.stream, (float *)x, (long long)count, (float)value);
    return hip_check(hipGetLastError(), "fill");
}

int launch_aos_to_soa(const feh_plan &p, const void *aos, void *soa) {
    const int g = grid_for(p.N * p.dim * p.L);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL((k_transpose<double, true>), dim3(g), dim3(kThreads), 0, p.stream, (const double *)aos,
                           (double *)soa, (long long)p.N, p.dim, p.L);
    else
        hipLaunchKernelGGL((k_transpose<float, true>), dim3(g), dim3(kThreads), 0, p.stream, (const float *)aos,
                           (float *)soa, (long long)p.N, p.dim, p.L);
    return hip_check(hipGetLastError(), "aos->soa");
}

int launch_soa_to_aos(const feh_plan &p, const void *soa, void *aos) {
    const int g = grid_for(p.N * p.dim * p.L);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL((k_transpose<double, false>), dim3(g), dim3(kThreads), 0, p.stream, (const double *)soa,
                           (double *)aos, (long long)p.N, p.dim, p.L);
    else
        hipLaunchKernelGGL((k_transpose<float, false>), dim3(g), dim3(kThreads), 0, p.stream, (const float *)soa,
                           (float *)aos, (long long)p.N, p.dim, p.L);
    return hip_check(hipGetLastError(), "soa->aos");
}

int launch_init_state(const feh_plan &p, LcState *st, int n_load) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(kMaxLoad), 0, p.stream, st, n_load);
    return hip_check(hipGetLastError(), "init state");
}

int launch_finish_rho(const feh_plan &p, LcState *st, const double *partial, int nparts, int mode, double tol,
                      int max_iter) {
    const int ref_too = mode >= 10 ? 1 : 0;
    hipLaunchKernelGGL(k_finish_rho, dim3(p.L), dim3(kThreads), 0, p.stream, st, partial, nparts, (int)p.part_stride,
                       mode % 10, ref_too, tol, max_iter);
    return hip_check(hipGetLastError(), "finish rho");
}

int launch_finish_rho_stride(const feh_plan &p, LcState *st, const double *partial, int nparts, int stride,
                             int mode, double tol, int max_iter) {
    const int ref_too = mode >= 10 ? 1 : 0;
    hipLaunchKernelGGL(k_finish_rho, dim3(p.L), dim3(kThreads), 0, p.stream, st, partial, nparts, stride, mode % 10,
                       ref_too, tol, max_iter);
    return hip_check(hipGetLastError(), "finish rho");
}

int launch_finish_pq_stride(const feh_plan &p, LcState *st, const double *partial, int nparts, int stride) {
    hipLaunchKernelGGL(k_finish_pq, dim3(p.L), dim3(kThreads), 0, p.stream, st, partial, nparts, stride);
    return hip_check(hipGetLastError(), "finish pq");
}

int launch_finish_pq(const feh_plan &p, LcState *st, const double *partial, int nparts) {
    hipLaunchKernelGGL(k_finish_pq, dim3(p.L), dim3(kThreads), 0, p.stream, st, partial, nparts, (int)p.part_stride);
    return hip_check(hipGetLastError(), "finish pq");
}

int launch_finalize_u(const feh_plan &p, void *u, const void *pv, const LcState *st) {
    const long long per = p.N * p.dim;
    const int g = grid_for(per * p.L);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_finalize_u<double>, dim3(g), dim3(kThreads), 0, p.stream, (double *)u, (const double *)pv,
                           st, per, p.L);
    else
        hipLaunchKernelGGL(k_finalize_u<float>, dim3(g), dim3(kThreads), 0, p.stream, (float *)u, (const float *)pv,
                           st, per, p.L);
    hipLaunchKernelGGL(k_clear_pending, dim3(1), dim3(kMaxLoad), 0, p.stream, (LcState *)st, p.L);
    return hip_check(hipGetLastError(), "finalize u");
}

int launch_material_lame(const feh_plan &p, const void *lam, const void *mu, int *flag) {
    const int g = grid_for(p.N * p.nbatch);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_mat_lame<double>, dim3(g), dim3(kThreads), 0, p.stream, (const double *)lam,
                           (const double *)mu, p.ptr<double>(p.off_lam), p.ptr<double>(p.off_mu), (long long)p.N * p.nbatch,
                           p.dim, flag);
    else
        hipLaunchKernelGGL(k_mat_lame<float>, dim3(g), dim3(kThreads), 0, p.stream, (const float *)lam,
                           (const float *)mu, p.ptr<float>(p.off_lam), p.ptr<float>(p.off_mu), (long long)p.N * p.nbatch, p.dim,
                           flag);
    return hip_check(hipGetLastError(), "material lame");
}

int launch_material_phases(const feh_plan &p, const int32_t *phase, const double *tab, int n_phase, int *flag) {
    const int g = grid_for(p.N * p.nbatch);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_mat_phases_d, dim3(g), dim3(kThreads), 0, p.stream, phase, tab, n_phase,
                           p.ptr<double>(p.off_lam), p.ptr<double>(p.off_mu), (long long)p.N * p.nbatch, flag);
    else
        hipLaunchKernelGGL(k_mat_phases_f, dim3(g), dim3(kThreads), 0, p.stream, phase, tab, n_phase,
                           p.ptr<float>(p.off_lam), p.ptr<float>(p.off_mu), (long long)p.N * p.nbatch, flag);
    return hip_check(hipGetLastError(), "material phases");
}

int launch_material_field(const feh_plan &p, const void *E, double nu, int *flag) {
    const double cl = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double cm = 1.0 / (2.0 * (1.0 + nu));
    const int g = grid_for(p.N * p.nbatch);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_mat_field<double>, dim3(g), dim3(kThreads), 0, p.stream, (const double *)E,
                           p.ptr<double>(p.off_lam), p.ptr<double>(p.off_mu), (long long)p.N * p.nbatch, cl, cm, flag);
    else
        hipLaunchKernelGGL(k_mat_field<float>, dim3(g), dim3(kThreads), 0, p.stream, (const float *)E,
                           p.ptr<float>(p.off_lam), p.ptr<float>(p.off_mu), (long long)p.N * p.nbatch, cl, cm, flag);
    return hip_check(hipGetLastError(), "material field");
}

int launch_remove_mean(const feh_plan &p, void *x, double *partial, double *mean) {
    long long nb = (p.N + kThreads - 1) / kThreads;
    if (nb > 512) nb = 512;
    const int nf = p.L * p.dim;
    const dim3 g((unsigned)nb, nf);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_mean_partial_d, g, dim3(kThreads), 0, p.stream, (const double *)x, (long long)p.N, (int)nb,
                           partial);
    else
        hipLaunchKernelGGL(k_mean_partial_f, g, dim3(kThreads), 0, p.stream, (const float *)x, (long long)p.N, (int)nb,
                           partial);
    hipLaunchKernelGGL(k_mean_finish, dim3(nf), dim3(kThreads), 0, p.stream, partial, (int)nb, mean, 1.0 / (double)p.N);
    const int gg = grid_for(p.N * nf);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_sub_mean<double>, dim3(gg), dim3(kThreads), 0, p.stream, (double *)x, (long long)p.N, nf,
                           mean);
    else
        hipLaunchKernelGGL(k_sub_mean<float>, dim3(gg), dim3(kThreads), 0, p.stream, (float *)x, (long long)p.N, nf,
                           mean);
    return hip_check(hipGetLastError(), "remove mean");
}

int launch_spec_to_numpy(const feh_plan &p, const void *spec, void *out, bool to_numpy) {
    const int g = grid_for(p.Nspec * p.dim * p.L);
    if (p.prec == FEH_FP64)
        hipLaunchKernelGGL(k_spec_numpy<double>, dim3(g), dim3(kThreads), 0, p.stream, (const Cx<double> *)spec,
                           (Cx<double> *)out, (long long)p.Nspec, p.dim, p.L, to_numpy ? 1 : 0);
    else
        hipLaunchKernelGGL(k_spec_numpy<float>, dim3(g), dim3(kThreads), 0, p.stream, (const Cx<float> *)spec,
                           (Cx<float> *)out, (long long)p.Nspec, p.dim, p.L, to_numpy ? 1 : 0);
    return hip_check(hipGetLastError(), "spectrum layout");
}

}  // namespace feh
