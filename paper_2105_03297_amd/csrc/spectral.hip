// Projected conjugate gradients in strain space with a choice of discrete
// derivative.
//
// Sec. "Discrete projection" builds the compatibility projection from the
// Fourier symbol of a discrete derivative; the derivatives offered here are
// those of Secs. "Finite differences" (forward and central), "Least squares"
// (2D), "Linear finite elements" (the FE gradient, n_e evaluation points per
// voxel), the Fourier derivative of Eq. original-G and the two-point Fourier
// derivative of the two-point appendix (2D).
//
// The unknown is the strain fluctuation itself, one symmetric D x D tensor per
// evaluation point T (n_e points per voxel), and CG runs on
//     A e~ = G(C : e~),  b = -G(C : Ebar),  e~_0 = 0,
// with the Euclidean (Frobenius, equal point weights) inner product (Sec.
// "Compatibility projection": solvers started from a compatible field stay
// compatible).  Per wavevector the operator of the small-strain appendix
// reduces to
//     G(s)_T = sym(D_T (x) w),  w = M^-1 V,  V = sum_L s_L . conj(D_L),
//     M = 1/2 (S I + sum_L D_L D_L^H),  S = sum_L |D_L|^2
// (the appendix's h = (I + sum_T g_TT)^-1 equals 2 S M^-1).  G is invariant
// under a common scaling of the symbol, so the kernels normalise it to S = 1;
// where it vanishes (k = 0, which carries the mean strain, and on even grids
// the modes where central differences or the least-squares stencil lose all
// directions) the mode is projected out.
//
// Real fields are transformed with the half-spectrum r2c/c2r pair, which
// keeps the Hermitian part of a spectrum.  For the stencil derivatives the
// symbol is itself Hermitian (D(-k) = conj D(k)); the Fourier derivatives take
// k at the Nyquist index as -pi/h (the appendix's wavevector range), which
// breaks that symmetry, and there the kernel applies the Hermitian part
// 1/2 (G(k) + conj G(-k)) of the operator, i.e. the real part of the complex
// result.
//
// Layouts: real fields [L][C][N] with C = n_e * nsym components per voxel
// (symmetric components xx, yy, (zz, yz, xz,) xy per point); spectra
// [L][C][n0][(n1)][nh] (the FFT kernels run the L * C scalar fields as one
// batch).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "symbols.hpp"

namespace feh {
namespace {

// ---------------------------------------------------------------------------
// device: field kernels
// ---------------------------------------------------------------------------
template <typename T>
struct PK {
    T *x, *r, *p, *q;           // [L][C][N]; q doubles as the stress buffer
    const T *lam, *mu;          // [N]
    const double *Ebar;         // [L][D][D]
    void *spec;                 // [L][C][Nspec] complex
    double *partial;            // [L][kVecBlocks] (or [quantities][kPostBlocks])
    LcState *st;
    long long N, Nspec;
    int L, C, ne;
};

template <int DIM>
__device__ __forceinline__ void ebar_sym(const double *E, double (&eb)[nsym(DIM)]) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = i; j < DIM; ++j) eb[sidx<DIM>(i, j)] = E[i * DIM + j];
}

// q = C : e at every point, e = Ebar (RHS) or e = p after p = r + beta p
template <typename T, int DIM, bool RHS>
__global__ __launch_bounds__(kThreads) void k_sc_stress(PK<T> a) {
    constexpr int NS = nsym(DIM);
    const long long total = a.N * a.L;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < total; i += (long long)gridDim.x * kThreads) {
        const int l = (int)(i / a.N);
        const long long v = i - (long long)l * a.N;
        if (!RHS && !a.st[l].active) continue;
        const double lam = double(a.lam[v]), mu2 = 2.0 * double(a.mu[v]);
        const long long base = (long long)l * a.C * a.N + v;
        double eb[NS];
        if (RHS) ebar_sym<DIM>(a.Ebar + l * DIM * DIM, eb);
        const double beta = RHS ? 0.0 : a.st[l].beta;
        for (int t = 0; t < a.ne; ++t) {
            double e[NS];
            #pragma unroll
            for (int c = 0; c < NS; ++c) {
                if (RHS) {
                    e[c] = eb[c];
                } else {
                    const long long o = base + (long long)(t * NS + c) * a.N;
                    const T pv = T(double(a.r[o]) + beta * double(a.p[o]));
                    a.p[o] = pv;
                    e[c] = double(pv);
                }
            }
            double tr = 0.0;
            #pragma unroll
            for (int c = 0; c < DIM; ++c) tr += e[c];
            #pragma unroll
            for (int c = 0; c < NS; ++c)
                a.q[base + (long long)(t * NS + c) * a.N] = T((c < DIM ? lam * tr : 0.0) + mu2 * e[c]);
        }
    }
}

// Per wavevector: s -> sym(D_T (x) M^-1 sum_L s_L . conj(D_L)) for every
// active load case (Hermitian part at Nyquist indices of the Fourier
// derivatives).
template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(kThreads) void k_sc_project(PK<T> a, SymArgs sa) {
    constexpr int NS = nsym(DIM);
    constexpr int NE = Pts<DIM, KIND>::NE;
    constexpr bool FOUR = KIND == K_FOURIER || KIND == K_FOURIER2;
    Cx<T> *spec = static_cast<Cx<T> *>(a.spec);
    const long long cs = a.Nspec;  // component stride
    for (long long k = blockIdx.x * (long long)kThreads + threadIdx.x; k < a.Nspec; k += (long long)gridDim.x * kThreads) {
        using CT = Cx<T>;
        // symbol and inverse in FP64, rounded once to the plan precision
        CT Dt[NE][DIM], D2t[FOUR ? NE : 1][DIM];
        T Md[DIM], M2d[FOUR ? DIM : 1];
        CT Mo[3], M2o[FOUR ? 3 : 1];
        bool two = false, ok;
        {
            C64 D[NE][DIM];
            bool nyq = false;
            double Id[DIM];
            C64 Io[3];
            ok = symbol_at<DIM, KIND, false>(sa, k, D, nyq);
            if (ok) metric_inverse<DIM, NE>(D, Id, Io);
            #pragma unroll
            for (int t = 0; t < NE; ++t)
                #pragma unroll
                for (int x = 0; x < DIM; ++x) Dt[t][x] = CT{T(D[t][x].x), T(D[t][x].y)};
            #pragma unroll
            for (int x = 0; x < DIM; ++x) Md[x] = T(ok ? Id[x] : 0.0);
            #pragma unroll
            for (int u = 0; u < 3; ++u) Mo[u] = ok ? CT{T(Io[u].x), T(Io[u].y)} : CT{T(0), T(0)};
            if constexpr (FOUR) {
                bool dummy;
                two = ok && nyq;
                if (two) {
                    symbol_at<DIM, KIND, true>(sa, k, D, dummy);
                    metric_inverse<DIM, NE>(D, Id, Io);
                    #pragma unroll
                    for (int t = 0; t < NE; ++t)
                        #pragma unroll
                        for (int x = 0; x < DIM; ++x) D2t[t][x] = CT{T(D[t][x].x), T(D[t][x].y)};
                    #pragma unroll
                    for (int x = 0; x < DIM; ++x) M2d[x] = T(Id[x]);
                    #pragma unroll
                    for (int u = 0; u < 3; ++u) M2o[u] = CT{T(Io[u].x), T(Io[u].y)};
                }
            }
        }
        // w = M^-1 V from the diagonal and upper triangle
        auto apply = [](const T (&md)[DIM], const CT (&mo)[3], const CT (&V)[DIM], CT (&w)[DIM]) {
            if constexpr (DIM == 2) {
                w[0] = cadd(cscale(V[0], md[0]), cmul(mo[0], V[1]));
                w[1] = cadd(cmulc(V[0], mo[0]), cscale(V[1], md[1]));
            } else {
                w[0] = cadd(cadd(cscale(V[0], md[0]), cmul(mo[0], V[1])), cmul(mo[1], V[2]));
                w[1] = cadd(cadd(cmulc(V[0], mo[0]), cscale(V[1], md[1])), cmul(mo[2], V[2]));
                w[2] = cadd(cadd(cmulc(V[0], mo[1]), cmulc(V[1], mo[2])), cscale(V[2], md[2]));
            }
        };
        const T half = T(0.5);
        for (int l = 0; l < a.L; ++l) {
            // keep this load case's spectrum loads from being hoisted above
            // the symbol evaluation (register pressure)
            asm volatile("" ::: "memory");
            if (!a.st[l].active) continue;
            CT *sp = spec + (long long)l * a.C * cs + k;
            if (!ok) {
                #pragma unroll
                for (int c = 0; c < NE * NS; ++c) sp[c * cs] = CT{T(0), T(0)};
                continue;
            }
            CT V[DIM], V2[DIM];
            #pragma unroll
            for (int x = 0; x < DIM; ++x) V[x] = V2[x] = CT{T(0), T(0)};
            #pragma unroll
            for (int t = 0; t < NE; ++t)
                #pragma unroll
                for (int x = 0; x < DIM; ++x)
                    #pragma unroll
                    for (int y = 0; y < DIM; ++y) {
                        const CT sv = sp[(t * NS + sidx<DIM>(x, y)) * cs];
                        V[x] = cadd(V[x], cmulc(sv, Dt[t][y]));
                        if constexpr (FOUR)
                            if (two) V2[x] = cadd(V2[x], cmulc(sv, D2t[t][y]));
                    }
            CT w[DIM], w2[DIM];
            apply(Md, Mo, V, w);
            if constexpr (FOUR)
                if (two) apply(M2d, M2o, V2, w2);
            #pragma unroll
            for (int t = 0; t < NE; ++t)
                #pragma unroll
                for (int x = 0; x < DIM; ++x)
                    #pragma unroll
                    for (int y = x; y < DIM; ++y) {
                        CT e = cscale(cadd(cmul(Dt[t][x], w[y]), cmul(Dt[t][y], w[x])), half);
                        if constexpr (FOUR)
                            if (two) {
                                const CT e2 = cscale(cadd(cmul(D2t[t][x], w2[y]), cmul(D2t[t][y], w2[x])), half);
                                e = cscale(cadd(e, e2), half);
                            }
                        sp[(t * NS + sidx<DIM>(x, y)) * cs] = e;
                    }
        }
    }
}

// MODE 0: partial of p.q; MODE 1: r = p = -q, x = 0, partial of r.r (start);
// MODE 2: x += alpha p, r -= alpha q, partial of r.r.  Frobenius weights:
// off-diagonal components count twice.
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(kThreads) void k_sc_vec(PK<T> a) {
    constexpr int NS = nsym(DIM);
    __shared__ double red[kThreads / 64];
    const int l = blockIdx.y;
    if (MODE != 1 && !a.st[l].active) return;
    const double alpha = MODE == 2 ? a.st[l].alpha : 0.0;
    double acc = 0.0;
    for (int c = 0; c < a.C; ++c) {
        const double wgt = (c % NS) < DIM ? 1.0 : 2.0;
        const long long off = ((long long)l * a.C + c) * a.N;
        T *xx = a.x + off, *rr = a.r + off, *pp = a.p + off;
        const T *qq = a.q + off;
        double s = 0.0;
        for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < a.N; i += (long long)gridDim.x * kThreads) {
            if (MODE == 0) {
                s += double(pp[i]) * double(qq[i]);
            } else if (MODE == 1) {
                const T rv = T(-double(qq[i]));
                rr[i] = rv;
                pp[i] = rv;
                xx[i] = T(0);
                s += double(rv) * double(rv);
            } else {
                xx[i] = T(double(xx[i]) + alpha * double(pp[i]));
                const T rv = T(double(rr[i]) - alpha * double(qq[i]));
                rr[i] = rv;
                s += double(rv) * double(rv);
            }
        }
        acc += wgt * s;
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) a.partial[(long long)l * gridDim.x + blockIdx.x] = tot;
}

// Post-processing with e = Ebar + x.  Quantity q < L * NS: the stress
// component q % NS of load case q / NS summed over all points (the strain
// output, if any, is written by the blocks of component 0); then the pairs
// l <= m of the energy e_l : C : e_m.
template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_sc_post(PK<T> a, T *strain) {
    constexpr int NS = nsym(DIM);
    __shared__ double red[kThreads / 64];
    const int q = blockIdx.y;
    int l = 0, m = -1, comp = 0;
    if (q < a.L * NS) {
        l = q / NS;
        comp = q % NS;
    } else {
        int rem = q - a.L * NS;
        while (rem >= a.L - l) {
            rem -= a.L - l;
            ++l;
        }
        m = l + rem;
    }
    double ebl[NS], ebm[NS];
    ebar_sym<DIM>(a.Ebar + l * DIM * DIM, ebl);
    ebar_sym<DIM>(a.Ebar + (m < 0 ? l : m) * DIM * DIM, ebm);
    double acc = 0.0;
    for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)gridDim.x * kThreads) {
        const double lam = double(a.lam[v]), mu2 = 2.0 * double(a.mu[v]);
        for (int t = 0; t < a.ne; ++t) {
            double e[NS];
            #pragma unroll
            for (int c = 0; c < NS; ++c) e[c] = ebl[c] + double(a.x[((long long)l * a.C + t * NS + c) * a.N + v]);
            double tr = 0.0;
            #pragma unroll
            for (int c = 0; c < DIM; ++c) tr += e[c];
            if (m < 0) {
                acc += (comp < DIM ? lam * tr : 0.0) + mu2 * e[comp];
                if (strain && comp == 0) {
                    T *o = strain + (((long long)l * a.N + v) * a.ne + t) * DIM * DIM;
                    #pragma unroll
                    for (int i = 0; i < DIM; ++i)
                        #pragma unroll
                        for (int j = 0; j < DIM; ++j) o[i * DIM + j] = T(e[sidx<DIM>(i, j)]);
                }
            } else {
                double f[NS];
                #pragma unroll
                for (int c = 0; c < NS; ++c) f[c] = ebm[c] + double(a.x[((long long)m * a.C + t * NS + c) * a.N + v]);
                double tf = 0.0, dd = 0.0;
                #pragma unroll
                for (int c = 0; c < NS; ++c) {
                    if (c < DIM) tf += f[c];
                    dd += (c < DIM ? 1.0 : 2.0) * e[c] * f[c];
                }
                acc += lam * tr * tf + mu2 * dd;
            }
        }
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) a.partial[(long long)q * gridDim.x + blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_sc_reduce(const double *part, int nblk, double *out, double scale) {
    __shared__ double red[kThreads / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) v += part[(long long)blockIdx.x * nblk + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}


// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct Layout {
    size_t x, r, p, q, spec, ebar, state, part, sums, total;
};

int num_quantities(int L, int dim) { return L * nsym(dim) + L * (L + 1) / 2; }

Layout make_layout(const feh_plan &p, int ne) {
    const size_t C = (size_t)ne * nsym(p.dim);
    const size_t vec = (size_t)p.L * C * p.N * p.rsize;
    Layout Lo{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = (o + b + 255) & ~size_t(255);
        return at;
    };
    Lo.x = take(vec);
    Lo.r = take(vec);
    Lo.p = take(vec);
    Lo.q = take(vec);
    Lo.spec = take((size_t)p.L * C * p.Nspec * 2 * p.rsize);
    Lo.ebar = take((size_t)p.L * 9 * sizeof(double));
    Lo.state = take((size_t)p.L * sizeof(LcState));
    const size_t np = std::max((size_t)p.L * kVecBlocks, (size_t)num_quantities(p.L, p.dim) * kPostBlocks);
    Lo.part = take(np * sizeof(double));
    Lo.sums = take((size_t)num_quantities(p.L, p.dim) * sizeof(double));
    Lo.total = o;
    return Lo;
}

struct Run {
    feh_plan &p;
    feh_plan fp;  // the plan seen by the FFT kernels: L * C scalar fields
    int kind, ne, C;
    Layout Lo;
    char *w;
};

template <typename T, int DIM, int KIND>
int launch_project(const feh_plan &p, const PK<T> &a, const SymArgs &sa) {
    hipLaunchKernelGGL((k_sc_project<T, DIM, KIND>), dim3(grid_of(p.Nspec)), dim3(kThreads), 0, p.stream, a, sa);
    return hip_check(hipGetLastError(), "strain-space projection");
}

template <typename T, int DIM>
int project_dispatch(const feh_plan &p, int kind, const PK<T> &a, const SymArgs &sa) {
    switch (kind) {
    case K_FE: return launch_project<T, DIM, K_FE>(p, a, sa);
    case K_FD: return launch_project<T, DIM, K_FD>(p, a, sa);
    case K_CD: return launch_project<T, DIM, K_CD>(p, a, sa);
    case K_FOURIER: return launch_project<T, DIM, K_FOURIER>(p, a, sa);
    default:
        if constexpr (DIM == 2) {
            if (kind == K_LS) return launch_project<T, 2, K_LS>(p, a, sa);
            if (kind == K_FOURIER2) return launch_project<T, 2, K_FOURIER2>(p, a, sa);
        }
        return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
    }
}

template <typename T, int DIM>
int solve_t(Run &R, double tol, int max_iter, void *strain, std::vector<double> &sums, std::vector<LcState> &hs) {
    feh_plan &p = R.p;
    PK<T> a{};
    a.x = reinterpret_cast<T *>(R.w + R.Lo.x);
    a.r = reinterpret_cast<T *>(R.w + R.Lo.r);
    a.p = reinterpret_cast<T *>(R.w + R.Lo.p);
    a.q = reinterpret_cast<T *>(R.w + R.Lo.q);
    a.spec = R.w + R.Lo.spec;
    a.Ebar = reinterpret_cast<const double *>(R.w + R.Lo.ebar);
    a.st = reinterpret_cast<LcState *>(R.w + R.Lo.state);
    a.partial = reinterpret_cast<double *>(R.w + R.Lo.part);
    a.lam = p.ptr<const T>(p.off_lam);
    a.mu = p.ptr<const T>(p.off_mu);
    a.N = p.N;
    a.Nspec = p.Nspec;
    a.L = p.L;
    a.C = R.C;
    a.ne = R.ne;
    const SymArgs sa = make_sym_args(p, R.kind);
    // q <- G(q): the FFT pair over the L * C scalar fields with the projection between
    auto project = [&]() -> int {
        FftArgs fa;
        fa.comps = 1;
        fa.spec = a.spec;
        fa.r = a.q;
        CK(launch_forward_last(R.fp, fa));
        if (DIM == 3) CK(launch_middle(R.fp, fa, false));
        CK(launch_first_plain(R.fp, fa, false));
        CK(project_dispatch<T, DIM>(p, R.kind, a, sa));
        CK(launch_first_plain(R.fp, fa, true));
        if (DIM == 3) CK(launch_middle(R.fp, fa, true));
        fa.z = a.q;
        fa.out_scale = 1.0 / (double)p.N;
        return launch_inverse_last(R.fp, fa);
    };
    auto vec = [&](int mode) -> int {
        const dim3 g(kVecBlocks, p.L);
        if (mode == 0) hipLaunchKernelGGL((k_sc_vec<T, DIM, 0>), g, dim3(kThreads), 0, p.stream, a);
        else if (mode == 1) hipLaunchKernelGGL((k_sc_vec<T, DIM, 1>), g, dim3(kThreads), 0, p.stream, a);
        else hipLaunchKernelGGL((k_sc_vec<T, DIM, 2>), g, dim3(kThreads), 0, p.stream, a);
        return hip_check(hipGetLastError(), "strain-space CG vector kernel");
    };
    const int gs = grid_of(p.N * p.L);
    // start: x = 0, r = p = b = -G(C : Ebar), rho = r.r (also the reference)
    CK(launch_init_state(p, a.st, p.L));
    hipLaunchKernelGGL((k_sc_stress<T, DIM, true>), dim3(gs), dim3(kThreads), 0, p.stream, a);
    CK(hip_check(hipGetLastError(), "strain-space stress"));
    CK(project());
    CK(vec(1));
    CK(launch_finish_rho_stride(p, a.st, a.partial, kVecBlocks, kVecBlocks, 11, tol, max_iter));
    hs.resize(p.L);
    int done = 0, chunk = 4;
    while (done < max_iter) {
        CK(hip_check(hipMemcpyAsync(hs.data(), a.st, p.L * sizeof(LcState), hipMemcpyDeviceToHost, p.stream),
                     "read CG state"));
        CK(hip_check(hipStreamSynchronize(p.stream), "strain-space CG"));
        bool any = false;
        for (const LcState &s : hs) any = any || s.active;
        if (!any) break;
        const int c = std::min(chunk, max_iter - done);
        for (int it = 0; it < c; ++it) {
            // p = r + beta p, q = G(C : p), alpha = r.r / p.q, x += alpha p, r -= alpha q
            hipLaunchKernelGGL((k_sc_stress<T, DIM, false>), dim3(gs), dim3(kThreads), 0, p.stream, a);
            CK(hip_check(hipGetLastError(), "strain-space stress"));
            CK(project());
            CK(vec(0));
            CK(launch_finish_pq_stride(p, a.st, a.partial, kVecBlocks, kVecBlocks));
            CK(vec(2));
            CK(launch_finish_rho_stride(p, a.st, a.partial, kVecBlocks, kVecBlocks, 2, tol, max_iter));
        }
        done += c;
        if (chunk < 16) chunk *= 2;
    }
    const int nq = num_quantities(p.L, DIM);
    hipLaunchKernelGGL((k_sc_post<T, DIM>), dim3(kPostBlocks, nq), dim3(kThreads), 0, p.stream, a,
                       static_cast<T *>(strain));
    CK(hip_check(hipGetLastError(), "strain-space post-processing"));
    double *dsum = reinterpret_cast<double *>(R.w + R.Lo.sums);
    hipLaunchKernelGGL(k_sc_reduce, dim3(nq), dim3(kThreads), 0, p.stream, a.partial, kPostBlocks, dsum,
                       1.0 / ((double)p.N * R.ne));
    CK(hip_check(hipGetLastError(), "strain-space reduction"));
    sums.resize(nq);
    CK(hip_check(hipMemcpyAsync(sums.data(), dsum, nq * sizeof(double), hipMemcpyDeviceToHost, p.stream), "read sums"));
    CK(hip_check(hipMemcpyAsync(hs.data(), a.st, p.L * sizeof(LcState), hipMemcpyDeviceToHost, p.stream),
                 "read CG state"));
    return hip_check(hipStreamSynchronize(p.stream), "strain-space CG");
}

int check_kind(const feh_plan *p, int kind, int &ne) {
    if (!p) return set_error(FEH_EINVAL, "null plan");
    ne = points_of(kind, p->dim);
    if (ne < 1) return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
    return FEH_OK;
}

}  // namespace
}  // namespace feh

using namespace feh;

extern "C" {

int feh_strain_cg_points(int kind, int dim, int *n_points) {
    if (!n_points) return set_error(FEH_EINVAL, "null output");
    const int ne = points_of(kind, dim);
    if (ne < 1) return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
    *n_points = ne;
    return FEH_OK;
}

int feh_strain_cg_workspace_bytes(const feh_plan *plan, int kind, size_t *bytes) {
    int ne = 0;
    CK(check_kind(plan, kind, ne));
    if (!bytes) return set_error(FEH_EINVAL, "null output");
    *bytes = make_layout(*plan, ne).total;
    return FEH_OK;
}

int feh_strain_cg_solve(feh_plan *plan, int kind, const double *Ebar_host, double tol, int max_iter, void *work_dev,
                        size_t work_bytes, void *strain_dev, double *stress_mean_host, double *energy_host,
                        feh_report *report_host) {
    try {
        const double t0 = wall_seconds();
        int ne = 0;
        CK(check_kind(plan, kind, ne));
        feh_plan &p = *plan;
        if (!p.ws) return set_error(FEH_ENOMEM, "workspace not set (feh_plan_set_workspace)");
        if (!p.material_set) return set_error(FEH_EINVAL, "material not set");
        if (p.nbatch != 1) return set_error(FEH_EINVAL, "strain-space CG takes plans of one microstructure");
        if (!Ebar_host) return set_error(FEH_EINVAL, "null Ebar");
        if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(FEH_EINVAL, "tol must be finite and >= 0");
        if (max_iter < 1) return set_error(FEH_EINVAL, "max_iter must be >= 1");
        const int D = p.dim;
        for (int l = 0; l < p.L; ++l)
            for (int i = 0; i < D; ++i)
                for (int j = 0; j < D; ++j) {
                    const double x = Ebar_host[(l * D + i) * D + j], y = Ebar_host[(l * D + j) * D + i];
                    if (!std::isfinite(x)) return set_error(FEH_EINVAL, "Ebar must be finite");
                    if (std::fabs(x - y) > 1e-12 * (std::fabs(x) + std::fabs(y)) + 1e-300)
                        return set_error(FEH_EINVAL, "Ebar must be symmetric");
                }
        const Layout Lo = make_layout(p, ne);
        if (!work_dev || work_bytes < Lo.total)
            return set_error(FEH_ENOMEM, "strain-space CG workspace missing or too small");
        if (reinterpret_cast<uintptr_t>(work_dev) % 256)
            return set_error(FEH_EINVAL, "workspace must be 256-byte aligned");
        const int C = ne * nsym(D);
        Run R{p, p, kind, ne, C, Lo, static_cast<char *>(work_dev)};
        R.fp.L = p.L * C;
        R.fp.prof_on = false;
        // the FFT launch grids count blocks in int: rows * L * C must fit
        if ((double)(p.N / p.n[D - 1]) * R.fp.L >= 2147483647.0)
            return set_error(FEH_ENOTSUP, "grid too large for the strain-space solver");
        std::vector<double> eb(Ebar_host, Ebar_host + (size_t)p.L * D * D);
        CK(hip_check(hipMemcpyAsync(R.w + Lo.ebar, eb.data(), eb.size() * sizeof(double), hipMemcpyHostToDevice,
                                    p.stream),
                     "upload Ebar"));
        CK(hip_check(hipStreamSynchronize(p.stream), "upload Ebar"));
        std::vector<double> sums;
        std::vector<LcState> hs;
        int rc;
        if (p.prec == FEH_FP64)
            rc = D == 3 ? solve_t<double, 3>(R, tol, max_iter, strain_dev, sums, hs)
                        : solve_t<double, 2>(R, tol, max_iter, strain_dev, sums, hs);
        else
            rc = D == 3 ? solve_t<float, 3>(R, tol, max_iter, strain_dev, sums, hs)
                        : solve_t<float, 2>(R, tol, max_iter, strain_dev, sums, hs);
        CK(rc);
        const int ns = nsym(D);
        if (stress_mean_host)
            for (int l = 0; l < p.L; ++l)
                for (int i = 0; i < D; ++i)
                    for (int j = 0; j < D; ++j)
                        stress_mean_host[((size_t)l * D + i) * D + j] =
                            sums[(size_t)l * ns + (D == 3 ? sidx<3>(i, j) : sidx<2>(i, j))];
        if (energy_host) {
            int k = 0;
            for (int l = 0; l < p.L; ++l)
                for (int m = l; m < p.L; ++m, ++k) {
                    const double v = sums[(size_t)p.L * ns + k];
                    energy_host[l * p.L + m] = v;
                    energy_host[m * p.L + l] = v;
                }
        }
        rc = FEH_OK;
        stamp_reports(report_host, p.L, t0);
        for (int l = 0; l < p.L; ++l) {
            if (report_host) {
                report_host[l].iterations = hs[l].iters;
                report_host[l].status = hs[l].status;
                report_host[l].rel_residual = hs[l].relres;
            }
            if (hs[l].status == FEH_EBREAKDOWN) rc = FEH_EBREAKDOWN;
            else if ((hs[l].status == FEH_ENOCONV || hs[l].active) && rc == FEH_OK) rc = FEH_ENOCONV;
        }
        if (rc == FEH_ENOCONV) return set_error(rc, "max_iter reached before the tolerance");
        if (rc == FEH_EBREAKDOWN) return set_error(rc, "CG breakdown (p.q <= 0 or not finite)");
        return FEH_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

}  // extern "C"
