// Finite-strain homogenization: Newton + projected CG on the deformation
// gradient with the gradient projection of a chosen discrete derivative.
//
// Sec. "Compatibility projection": the unknown is the deformation gradient F
// (one D x D tensor per evaluation point T, n_e points per voxel), its mean is
// the macroscopic Fbar, and equilibrium in weak form reads G P(F) = 0 with G
// the projection onto compatible (gradient) fields.  Per wavevector
// G_{i a b j} = delta_ij g_ab, g_ab = D_a conj(D_b) / sum_c |D_c|^2 over the
// derivative indices a = (T, alpha) (Eq. original-G, Eq. discrete_projection_op);
// with the symbol normalised to sum |D|^2 = 1 this is, row by row i,
//     (G s)_{T i alpha} = D_{T alpha} w_i,  w_i = sum_{L beta} conj(D_{L beta}) s_{L i beta}.
//
// Newton: each step solves G (K(F) : dF) = -G P(F) for a compatible dF by CG
// from dF = 0 (Euclidean inner product over all components, equal point
// weights), then F += dF; a load case stops when ||G P|| <= equil_tol ||P||
// before a step or ||dF|| <= newton_tol ||F|| after one.  The right-hand side
// is projected twice: G is idempotent, and one application leaves a rounding
// residue of order eps ||P|| outside the compatible subspace that would stall
// CG once ||G P|| << ||P||.  Load steps move Fbar linearly from I.
//
// Material: Saint Venant-Kirchhoff with the plan's per-voxel Lame constants,
// E = 1/2 (F^T F - I), S = lambda tr(E) I + 2 mu E, P = F S; the tangent is
// applied matrix-free, dP = X S + F (lambda tr(dE) I + 2 mu dE),
// dE = sym(F^T X), from F and X in registers (FP64 arithmetic).  lambda = mu = 0
// (vacuum) is allowed.
//
// Layouts: fields [L][C][N], C = n_e D^2, component (T D + i) D + alpha; the
// spectrum [L][C][n0][(n1)][nh]; the FFT passes run the L * C scalar fields as
// one batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "symbols.hpp"

namespace feh {
namespace {

template <typename T>
struct FSK {
    T *F, *dF, *r, *p, *q;      // [L][C][N]
    const T *lam, *mu;          // [N]
    void *spec;                 // [L][C][Nspec] complex
    double *partial;            // [2][L][kVecBlocks] or [L D^2][kPostBlocks]
    LcState *st;                // CG states (nullable: every load case)
    const int *nmask;           // Newton-active load cases
    const double *dFbar;        // [L][D][D] uniform increment of F
    long long N, Nspec;
    int L, C, ne;
};

template <int DIM>
struct Mat {
    double v[DIM][DIM];
};

template <int DIM>
__device__ __forceinline__ void pk2(const Mat<DIM> &F, double lam, double mu, Mat<DIM> &S) {
    double E[DIM][DIM];
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
            #pragma unroll
            for (int k = 0; k < DIM; ++k) s += F.v[k][i] * F.v[k][j];
            E[i][j] = 0.5 * (s - (i == j ? 1.0 : 0.0));
        }
    double tr = 0.0;
    #pragma unroll
    for (int i = 0; i < DIM; ++i) tr += E[i][i];
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) S.v[i][j] = (i == j ? lam * tr : 0.0) + 2.0 * mu * E[i][j];
}

template <int DIM>
__device__ __forceinline__ void matmul(const Mat<DIM> &A, const Mat<DIM> &B, Mat<DIM> &C) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
            #pragma unroll
            for (int k = 0; k < DIM; ++k) s += A.v[i][k] * B.v[k][j];
            C.v[i][j] = s;
        }
}

template <typename T, int DIM>
__device__ __forceinline__ void load_mat(const T *base, long long N, int t, Mat<DIM> &M) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) M.v[i][j] = double(base[(long long)((t * DIM + i) * DIM + j) * N]);
}

template <typename T, int DIM>
__device__ __forceinline__ void store_mat(T *base, long long N, int t, const Mat<DIM> &M) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) base[(long long)((t * DIM + i) * DIM + j) * N] = T(M.v[i][j]);
}

// F = I + dFbar (INIT) or F += dFbar, uniform per load case
template <typename T, int DIM, bool INIT>
__global__ __launch_bounds__(kThreads) void k_fs_uniform(FSK<T> a) {
    const long long per = (long long)a.C * a.N;
    const long long total = per * a.L;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < total; i += (long long)gridDim.x * kThreads) {
        const int l = (int)(i / per);
        const int c = (int)((i - l * per) / a.N);
        const int ij = c % (DIM * DIM);
        const double d = a.dFbar[l * DIM * DIM + ij];
        if (INIT) a.F[i] = T((ij / DIM == ij % DIM ? 1.0 : 0.0) + d);
        else a.F[i] = T(double(a.F[i]) + d);
    }
}

// q = P(F); partial sums of ||P||^2 per load case (grid: blocks x L)
template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_fs_pk1(FSK<T> a) {
    __shared__ double red[kThreads / 64];
    const int l = blockIdx.y;
    const long long off = (long long)l * a.C * a.N;
    double acc = 0.0;
    for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)gridDim.x * kThreads) {
        const double lam = double(a.lam[v]), mu = double(a.mu[v]);
        for (int t = 0; t < a.ne; ++t) {
            Mat<DIM> F, S, P;
            load_mat<T, DIM>(a.F + off + v, a.N, t, F);
            pk2<DIM>(F, lam, mu, S);
            matmul<DIM>(F, S, P);
            store_mat<T, DIM>(a.q + off + v, a.N, t, P);
            #pragma unroll
            for (int i = 0; i < DIM; ++i)
                #pragma unroll
                for (int j = 0; j < DIM; ++j) acc += P.v[i][j] * P.v[i][j];
        }
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) a.partial[(long long)l * gridDim.x + blockIdx.x] = tot;
}

// p = r + beta p, q = K(F) : p for the CG-active load cases
template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_fs_tangent(FSK<T> a) {
    const long long total = a.N * a.L;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < total; i += (long long)gridDim.x * kThreads) {
        const int l = (int)(i / a.N);
        const long long v = i - (long long)l * a.N;
        if (!a.st[l].active) continue;
        const double lam = double(a.lam[v]), mu = double(a.mu[v]);
        const double beta = a.st[l].beta;
        const long long off = (long long)l * a.C * a.N + v;
        for (int t = 0; t < a.ne; ++t) {
            Mat<DIM> F, X, S, dP;
            load_mat<T, DIM>(a.F + off, a.N, t, F);
            #pragma unroll
            for (int ii = 0; ii < DIM; ++ii)
                #pragma unroll
                for (int jj = 0; jj < DIM; ++jj) {
                    const long long o = off + (long long)((t * DIM + ii) * DIM + jj) * a.N;
                    const T pv = T(double(a.r[o]) + beta * double(a.p[o]));
                    a.p[o] = pv;
                    X.v[ii][jj] = double(pv);
                }
            pk2<DIM>(F, lam, mu, S);
            // dE = sym(F^T X), dS = lambda tr(dE) I + 2 mu dE
            Mat<DIM> dS;
            double tr = 0.0;
            #pragma unroll
            for (int ii = 0; ii < DIM; ++ii)
                #pragma unroll
                for (int jj = 0; jj < DIM; ++jj) {
                    double s = 0.0;
                    #pragma unroll
                    for (int k = 0; k < DIM; ++k) s += F.v[k][ii] * X.v[k][jj] + X.v[k][ii] * F.v[k][jj];
                    dS.v[ii][jj] = 0.5 * s;
                }
            #pragma unroll
            for (int ii = 0; ii < DIM; ++ii) tr += dS.v[ii][ii];
            #pragma unroll
            for (int ii = 0; ii < DIM; ++ii)
                #pragma unroll
                for (int jj = 0; jj < DIM; ++jj) dS.v[ii][jj] = (ii == jj ? lam * tr : 0.0) + 2.0 * mu * dS.v[ii][jj];
            // dP = X S + F dS
            #pragma unroll
            for (int ii = 0; ii < DIM; ++ii)
                #pragma unroll
                for (int jj = 0; jj < DIM; ++jj) {
                    double s = 0.0;
                    #pragma unroll
                    for (int k = 0; k < DIM; ++k) s += X.v[ii][k] * S.v[k][jj] + F.v[ii][k] * dS.v[k][jj];
                    dP.v[ii][jj] = s;
                }
            store_mat<T, DIM>(a.q + off, a.N, t, dP);
        }
    }
}

// Gradient projection per wavevector, row by row: out_{T i a} = D_{T a} w_i,
// w_i = sum_{L b} conj(D_{L b}) s_{L i b} (normalised symbol); the Hermitian
// part at Nyquist indices of the Fourier derivatives.  st == nullptr: every
// load case.
template <typename T, int DIM, int KIND>
__global__ __launch_bounds__(kThreads) void k_fs_project(FSK<T> a, SymArgs sa) {
    constexpr int NE = Pts<DIM, KIND>::NE;
    constexpr bool FOUR = KIND == K_FOURIER || KIND == K_FOURIER2;
    Cx<T> *spec = static_cast<Cx<T> *>(a.spec);
    const long long cs = a.Nspec;
    for (long long k = blockIdx.x * (long long)kThreads + threadIdx.x; k < a.Nspec; k += (long long)gridDim.x * kThreads) {
        C64 D[NE][DIM];
        bool nyq = false;
        const bool ok = symbol_at<DIM, KIND, false>(sa, k, D, nyq);
        C64 D2[NE][DIM];
        bool two = false;
        if constexpr (FOUR) {
            bool dummy;
            two = ok && nyq;
            if (two) symbol_at<DIM, KIND, true>(sa, k, D2, dummy);
        }
        for (int l = 0; l < a.L; ++l) {
            if (a.st && !a.st[l].active) continue;
            Cx<T> *sp = spec + (long long)l * a.C * cs + k;
            #pragma unroll
            for (int i = 0; i < DIM; ++i) {
                C64 w{0.0, 0.0}, w2{0.0, 0.0};
                if (ok) {
                    #pragma unroll
                    for (int t = 0; t < NE; ++t)
                        #pragma unroll
                        for (int b = 0; b < DIM; ++b) {
                            const Cx<T> s = sp[(long long)((t * DIM + i) * DIM + b) * cs];
                            const C64 sv{double(s.x), double(s.y)};
                            w = cadd(w, cmulc(sv, D[t][b]));
                            if constexpr (FOUR)
                                if (two) w2 = cadd(w2, cmulc(sv, D2[t][b]));
                        }
                }
                #pragma unroll
                for (int t = 0; t < NE; ++t)
                    #pragma unroll
                    for (int b = 0; b < DIM; ++b) {
                        C64 e = ok ? cmul(D[t][b], w) : C64{0.0, 0.0};
                        if constexpr (FOUR)
                            if (two) e = cscale(cadd(e, cmul(D2[t][b], w2)), 0.5);
                        sp[(long long)((t * DIM + i) * DIM + b) * cs] = Cx<T>{T(e.x), T(e.y)};
                    }
            }
        }
    }
}

// Vector kernels of CG on dF (all components weight 1; grid: blocks x L):
// MODE 0: partial p.q; MODE 1: r = p = -q, dF = 0, partial r.r;
// MODE 2: dF += alpha p, r -= alpha q, partial r.r;
// MODE 3: partial q.q (equilibrium norm, every load case).
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_fs_vec(FSK<T> a) {
    __shared__ double red[kThreads / 64];
    const int l = blockIdx.y;
    if ((MODE == 0 || MODE == 2) && !a.st[l].active) return;
    const double alpha = MODE == 2 ? a.st[l].alpha : 0.0;
    const long long per = (long long)a.C * a.N;
    const long long off = (long long)l * per;
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < per; i += (long long)gridDim.x * kThreads) {
        const long long o = off + i;
        if (MODE == 0) {
            acc += double(a.p[o]) * double(a.q[o]);
        } else if (MODE == 1) {
            const T rv = T(-double(a.q[o]));
            a.r[o] = rv;
            a.p[o] = rv;
            a.dF[o] = T(0);
            acc += double(rv) * double(rv);
        } else if (MODE == 2) {
            a.dF[o] = T(double(a.dF[o]) + alpha * double(a.p[o]));
            const T rv = T(double(a.r[o]) - alpha * double(a.q[o]));
            a.r[o] = rv;
            acc += double(rv) * double(rv);
        } else {
            acc += double(a.q[o]) * double(a.q[o]);
        }
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) a.partial[(long long)l * gridDim.x + blockIdx.x] = tot;
}

// F += dF for the Newton-active load cases; partials of ||dF||^2 and ||F||^2
// (after the update) in two consecutive [L][blocks] arrays.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fs_update(FSK<T> a) {
    __shared__ double red[kThreads / 64];
    const int l = blockIdx.y;
    const long long per = (long long)a.C * a.N;
    const long long off = (long long)l * per;
    const bool act = a.nmask[l] != 0;
    double s1 = 0.0, s2 = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < per; i += (long long)gridDim.x * kThreads) {
        const long long o = off + i;
        double f = double(a.F[o]);
        if (act) {
            const double d = double(a.dF[o]);
            f = double(T(f + d));
            a.F[o] = T(f);
            s1 += d * d;
        }
        s2 += f * f;
    }
    const double t1 = block_sum<kThreads>(s1, red);
    const double t2 = block_sum<kThreads>(s2, red);
    if (threadIdx.x == 0) {
        a.partial[(long long)l * gridDim.x + blockIdx.x] = t1;
        a.partial[((long long)a.L + l) * gridDim.x + blockIdx.x] = t2;
    }
}

// Post-processing: partial sums of P (quantity q = l D^2 + ij) and the
// optional F and P fields [L][N][n_e][D][D].
template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_fs_post(FSK<T> a, T *Fout, T *Pout) {
    __shared__ double red[kThreads / 64];
    const int q = blockIdx.y;
    const int l = q / (DIM * DIM), ij = q % (DIM * DIM);
    const long long off = (long long)l * a.C * a.N;
    double acc = 0.0;
    for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)gridDim.x * kThreads) {
        const double lam = double(a.lam[v]), mu = double(a.mu[v]);
        for (int t = 0; t < a.ne; ++t) {
            Mat<DIM> F, S, P;
            load_mat<T, DIM>(a.F + off + v, a.N, t, F);
            pk2<DIM>(F, lam, mu, S);
            matmul<DIM>(F, S, P);
            acc += P.v[ij / DIM][ij % DIM];
            if (ij == 0) {
                const long long o = (((long long)l * a.N + v) * a.ne + t) * DIM * DIM;
                #pragma unroll
                for (int i = 0; i < DIM; ++i)
                    #pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        if (Fout) Fout[o + i * DIM + j] = T(F.v[i][j]);
                        if (Pout) Pout[o + i * DIM + j] = T(P.v[i][j]);
                    }
            }
        }
    }
    const double tot = block_sum<kThreads>(acc, red);
    if (threadIdx.x == 0) a.partial[(long long)q * gridDim.x + blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_fs_reduce(const double *part, int nblk, double *out, double scale) {
    __shared__ double red[kThreads / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) v += part[(long long)blockIdx.x * nblk + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s * scale;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
struct FLayout {
    size_t F, dF, r, p, q, spec, dfbar, state, nmask, part, sums, total;
};

FLayout make_flayout(const feh_plan &p, int ne) {
    const size_t C = (size_t)ne * p.dim * p.dim;
    const size_t vec = (size_t)p.L * C * p.N * p.rsize;
    FLayout Lo{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = (o + b + 255) & ~size_t(255);
        return at;
    };
    Lo.F = take(vec);
    Lo.dF = take(vec);
    Lo.r = take(vec);
    Lo.p = take(vec);
    Lo.q = take(vec);
    Lo.spec = take((size_t)p.L * C * p.Nspec * 2 * p.rsize);
    Lo.dfbar = take((size_t)p.L * 9 * sizeof(double));
    Lo.state = take((size_t)p.L * sizeof(LcState));
    Lo.nmask = take((size_t)p.L * sizeof(int));
    const size_t np = std::max((size_t)2 * p.L * kVecBlocks, (size_t)p.L * 9 * kPostBlocks);
    Lo.part = take(np * sizeof(double));
    Lo.sums = take((size_t)2 * p.L * 9 * sizeof(double));
    Lo.total = o;
    return Lo;
}

struct FRun {
    feh_plan &p;
    feh_plan fp;  // the plan seen by the FFT kernels: L * C scalar fields
    int kind, ne, C;
    FLayout Lo;
    char *w;
};

template <typename T, int DIM, int KIND>
int fs_launch_project(const feh_plan &p, const FSK<T> &a, const SymArgs &sa) {
    hipLaunchKernelGGL((k_fs_project<T, DIM, KIND>), dim3(grid_of(p.Nspec)), dim3(kThreads), 0, p.stream, a, sa);
    return hip_check(hipGetLastError(), "gradient projection");
}

template <typename T, int DIM>
int fs_project_dispatch(const feh_plan &p, int kind, const FSK<T> &a, const SymArgs &sa) {
    switch (kind) {
    case K_FE: return fs_launch_project<T, DIM, K_FE>(p, a, sa);
    case K_FD: return fs_launch_project<T, DIM, K_FD>(p, a, sa);
    case K_CD: return fs_launch_project<T, DIM, K_CD>(p, a, sa);
    case K_FOURIER: return fs_launch_project<T, DIM, K_FOURIER>(p, a, sa);
    default:
        if constexpr (DIM == 2) {
            if (kind == K_LS) return fs_launch_project<T, 2, K_LS>(p, a, sa);
            if (kind == K_FOURIER2) return fs_launch_project<T, 2, K_FOURIER2>(p, a, sa);
        }
        return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
    }
}

struct FsParams {
    int n_steps, max_newton, max_cg;
    double newton_tol, equil_tol, cg_tol;
};

struct FsOut {
    std::vector<int> newton, cg, status;
    std::vector<double> rel_eq, rel_inc, pmean;
};

template <typename T, int DIM>
int fs_solve_t(FRun &R, const double *Fbar_host, const FsParams &prm, void *Fout, void *Pout, FsOut &out) {
    feh_plan &p = R.p;
    const int L = p.L;
    FSK<T> a{};
    a.F = reinterpret_cast<T *>(R.w + R.Lo.F);
    a.dF = reinterpret_cast<T *>(R.w + R.Lo.dF);
    a.r = reinterpret_cast<T *>(R.w + R.Lo.r);
    a.p = reinterpret_cast<T *>(R.w + R.Lo.p);
    a.q = reinterpret_cast<T *>(R.w + R.Lo.q);
    a.spec = R.w + R.Lo.spec;
    a.partial = reinterpret_cast<double *>(R.w + R.Lo.part);
    LcState *st = reinterpret_cast<LcState *>(R.w + R.Lo.state);
    int *nmask = reinterpret_cast<int *>(R.w + R.Lo.nmask);
    double *dfbar = reinterpret_cast<double *>(R.w + R.Lo.dfbar);
    double *sums = reinterpret_cast<double *>(R.w + R.Lo.sums);
    a.st = st;
    a.nmask = nmask;
    a.dFbar = dfbar;
    a.lam = p.ptr<const T>(p.off_lam);
    a.mu = p.ptr<const T>(p.off_mu);
    a.N = p.N;
    a.Nspec = p.Nspec;
    a.L = L;
    a.C = R.C;
    a.ne = R.ne;
    const SymArgs sa = make_sym_args(p, R.kind);
    const int gs = grid_of(p.N * L);
    const dim3 gv(kVecBlocks, L);
    // q <- G q over every load case (st == nullptr) or the CG-active ones
    auto project = [&](bool all) -> int {
        FSK<T> b = a;
        if (all) b.st = nullptr;
        FftArgs fa;
        fa.comps = 1;
        fa.spec = a.spec;
        fa.r = a.q;
        CK(launch_forward_last(R.fp, fa));
        if (DIM == 3) CK(launch_middle(R.fp, fa, false));
        CK(launch_first_plain(R.fp, fa, false));
        CK(fs_project_dispatch<T, DIM>(p, R.kind, b, sa));
        CK(launch_first_plain(R.fp, fa, true));
        if (DIM == 3) CK(launch_middle(R.fp, fa, true));
        fa.z = a.q;
        fa.out_scale = 1.0 / (double)p.N;
        return launch_inverse_last(R.fp, fa);
    };
    auto reduce = [&](int nq, int nblk, std::vector<double> &h) -> int {
        hipLaunchKernelGGL(k_fs_reduce, dim3(nq), dim3(kThreads), 0, p.stream, a.partial, nblk, sums, 1.0);
        CK(hip_check(hipGetLastError(), "reduce"));
        h.resize(nq);
        CK(hip_check(hipMemcpyAsync(h.data(), sums, nq * sizeof(double), hipMemcpyDeviceToHost, p.stream), "sums"));
        return hip_check(hipStreamSynchronize(p.stream), "finite strain");
    };
    out.newton.assign(L, 0);
    out.cg.assign(L, 0);
    out.status.assign(L, FEH_OK);
    out.rel_eq.assign(L, 0.0);
    out.rel_inc.assign(L, 0.0);
    std::vector<double> fb_prev(L * DIM * DIM, 0.0), fb(L * DIM * DIM), inc(L * DIM * DIM);
    for (int l = 0; l < L; ++l)
        for (int i = 0; i < DIM; ++i) fb_prev[(l * DIM + i) * DIM + i] = 1.0;
    std::vector<int> done(L), hmask(L);
    std::vector<LcState> hs(L);
    std::vector<double> h1, h2;
    for (int s = 1; s <= prm.n_steps; ++s) {
        for (int k = 0; k < L * DIM * DIM; ++k) {
            const int ij = k % (DIM * DIM);
            const double I = (ij / DIM == ij % DIM) ? 1.0 : 0.0;
            fb[k] = I + (double)s / prm.n_steps * (Fbar_host[k] - I);
            inc[k] = fb[k] - fb_prev[k];
        }
        fb_prev = fb;
        CK(hip_check(hipMemcpyAsync(dfbar, inc.data(), inc.size() * sizeof(double), hipMemcpyHostToDevice, p.stream),
                     "upload increment"));
        if (s == 1) hipLaunchKernelGGL((k_fs_uniform<T, DIM, true>), dim3(gs), dim3(kThreads), 0, p.stream, a);
        else hipLaunchKernelGGL((k_fs_uniform<T, DIM, false>), dim3(gs), dim3(kThreads), 0, p.stream, a);
        CK(hip_check(hipGetLastError(), "load step"));
        CK(hip_check(hipStreamSynchronize(p.stream), "load step"));
        std::fill(done.begin(), done.end(), 0);
        for (int it = 0; it < prm.max_newton; ++it) {
            // equilibrium residual G P(F)
            hipLaunchKernelGGL((k_fs_pk1<T, DIM>), gv, dim3(kThreads), 0, p.stream, a);
            CK(hip_check(hipGetLastError(), "stress"));
            CK(reduce(L, kVecBlocks, h1));  // ||P||^2
            CK(project(true));
            hipLaunchKernelGGL((k_fs_vec<T, 3>), gv, dim3(kThreads), 0, p.stream, a);
            CK(hip_check(hipGetLastError(), "norm"));
            CK(reduce(L, kVecBlocks, h2));  // ||G P||^2
            bool any = false;
            for (int l = 0; l < L; ++l) {
                if (done[l]) continue;
                const double nP = std::sqrt(h1[l]), nG = std::sqrt(h2[l]);
                out.rel_eq[l] = nP > 0.0 ? nG / nP : 0.0;
                if (nG <= prm.equil_tol * nP) done[l] = 1;
                any = any || !done[l];
            }
            if (!any) break;
            // second projection of the right-hand side, CG from dF = 0
            CK(project(true));
            for (int l = 0; l < L; ++l) {
                hs[l] = LcState{};
                hs[l].active = done[l] ? 0 : 1;
                hmask[l] = done[l] ? 0 : 1;
            }
            CK(hip_check(hipMemcpyAsync(st, hs.data(), L * sizeof(LcState), hipMemcpyHostToDevice, p.stream), "state"));
            CK(hip_check(hipMemcpyAsync(nmask, hmask.data(), L * sizeof(int), hipMemcpyHostToDevice, p.stream), "mask"));
            hipLaunchKernelGGL((k_fs_vec<T, 1>), gv, dim3(kThreads), 0, p.stream, a);
            CK(hip_check(hipGetLastError(), "cg start"));
            CK(launch_finish_rho_stride(p, st, a.partial, kVecBlocks, kVecBlocks, 11, prm.cg_tol, prm.max_cg));
            int cdone = 0, chunk = 4;
            while (cdone < prm.max_cg) {
                CK(hip_check(hipMemcpyAsync(hs.data(), st, L * sizeof(LcState), hipMemcpyDeviceToHost, p.stream),
                             "read CG state"));
                CK(hip_check(hipStreamSynchronize(p.stream), "finite strain CG"));
                bool cg_any = false;
                for (const LcState &x : hs) cg_any = cg_any || x.active;
                if (!cg_any) break;
                const int c = std::min(chunk, prm.max_cg - cdone);
                for (int k = 0; k < c; ++k) {
                    hipLaunchKernelGGL((k_fs_tangent<T, DIM>), dim3(gs), dim3(kThreads), 0, p.stream, a);
                    CK(hip_check(hipGetLastError(), "tangent"));
                    CK(project(false));
                    hipLaunchKernelGGL((k_fs_vec<T, 0>), gv, dim3(kThreads), 0, p.stream, a);
                    CK(hip_check(hipGetLastError(), "p.q"));
                    CK(launch_finish_pq_stride(p, st, a.partial, kVecBlocks, kVecBlocks));
                    hipLaunchKernelGGL((k_fs_vec<T, 2>), gv, dim3(kThreads), 0, p.stream, a);
                    CK(hip_check(hipGetLastError(), "cg update"));
                    CK(launch_finish_rho_stride(p, st, a.partial, kVecBlocks, kVecBlocks, 2, prm.cg_tol, prm.max_cg));
                }
                cdone += c;
                if (chunk < 16) chunk *= 2;
            }
            CK(hip_check(hipMemcpyAsync(hs.data(), st, L * sizeof(LcState), hipMemcpyDeviceToHost, p.stream),
                         "read CG state"));
            // F += dF; ||dF||, ||F||
            hipLaunchKernelGGL((k_fs_update<T>), gv, dim3(kThreads), 0, p.stream, a);
            CK(hip_check(hipGetLastError(), "newton update"));
            CK(reduce(2 * L, kVecBlocks, h1));
            for (int l = 0; l < L; ++l) {
                if (done[l]) continue;
                out.newton[l] += 1;
                out.cg[l] += hs[l].iters;
                const double nd = std::sqrt(h1[l]), nf = std::sqrt(h1[L + l]);
                out.rel_inc[l] = nf > 0.0 ? nd / nf : 0.0;
                if (nd <= prm.newton_tol * nf) done[l] = 1;
            }
        }
        for (int l = 0; l < L; ++l)
            if (!done[l]) out.status[l] = FEH_ENOCONV;
    }
    // post-processing: <P> and the fields
    const int nq = L * DIM * DIM;
    hipLaunchKernelGGL((k_fs_post<T, DIM>), dim3(kPostBlocks, nq), dim3(kThreads), 0, p.stream, a,
                       static_cast<T *>(Fout), static_cast<T *>(Pout));
    CK(hip_check(hipGetLastError(), "finite strain post-processing"));
    hipLaunchKernelGGL(k_fs_reduce, dim3(nq), dim3(kThreads), 0, p.stream, a.partial, kPostBlocks, sums,
                       1.0 / ((double)p.N * R.ne));
    CK(hip_check(hipGetLastError(), "reduce"));
    out.pmean.resize(nq);
    CK(hip_check(hipMemcpyAsync(out.pmean.data(), sums, nq * sizeof(double), hipMemcpyDeviceToHost, p.stream),
                 "read <P>"));
    return hip_check(hipStreamSynchronize(p.stream), "finite strain");
}

}  // namespace
}  // namespace feh

using namespace feh;

extern "C" {

int feh_finite_strain_workspace_bytes(const feh_plan *plan, int kind, size_t *bytes) {
    if (!plan || !bytes) return set_error(FEH_EINVAL, "null argument");
    const int ne = points_of(kind, plan->dim);
    if (ne < 1) return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
    *bytes = make_flayout(*plan, ne).total;
    return FEH_OK;
}

int feh_finite_strain_solve(feh_plan *plan, int kind, const double *Fbar_host, int n_steps, double newton_tol,
                            double equil_tol, double cg_tol, int max_newton, int max_cg, void *work_dev,
                            size_t work_bytes, void *F_dev, void *P_dev, double *P_mean_host,
                            feh_finite_report *report_host) {
    try {
        if (!plan) return set_error(FEH_EINVAL, "null plan");
        feh_plan &p = *plan;
        const int ne = points_of(kind, p.dim);
        if (ne < 1) return set_error(FEH_ENOTSUP, "derivative kind not defined in this dimension");
        if (kind == K_FOURIER || kind == K_FOURIER2) {
            // the Fourier derivative is ambiguous at the Nyquist wavevector of
            // an even axis, and its projection is exact on odd grids only; the
            // Newton iteration on the inexact one need not converge
            for (int a = 0; a < p.dim; ++a)
                if (p.n[a] % 2 == 0)
                    return set_error(FEH_ENOTSUP, "finite strain with a Fourier derivative needs odd grid sizes");
        }
        if (!p.ws) return set_error(FEH_ENOMEM, "workspace not set (feh_plan_set_workspace)");
        if (!p.material_set) return set_error(FEH_EINVAL, "material not set");
        if (p.nbatch != 1) return set_error(FEH_EINVAL, "finite strain takes plans of one microstructure");
        if (!Fbar_host) return set_error(FEH_EINVAL, "null Fbar");
        if (n_steps < 1 || max_newton < 1 || max_cg < 1) return set_error(FEH_EINVAL, "steps and iteration limits must be >= 1");
        for (double t : {newton_tol, equil_tol, cg_tol})
            if (!(t >= 0.0) || !std::isfinite(t)) return set_error(FEH_EINVAL, "tolerances must be finite and >= 0");
        const int D = p.dim;
        for (int k = 0; k < p.L * D * D; ++k)
            if (!std::isfinite(Fbar_host[k])) return set_error(FEH_EINVAL, "Fbar must be finite");
        for (int l = 0; l < p.L; ++l) {
            const double *A = Fbar_host + l * D * D;
            const double det = D == 2 ? A[0] * A[3] - A[1] * A[2]
                                      : A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                                            A[2] * (A[3] * A[7] - A[4] * A[6]);
            if (!(det > 0.0)) return set_error(FEH_EINVAL, "Fbar must have a positive determinant");
        }
        const FLayout Lo = make_flayout(p, ne);
        if (!work_dev || work_bytes < Lo.total) return set_error(FEH_ENOMEM, "finite-strain workspace missing or too small");
        if (reinterpret_cast<uintptr_t>(work_dev) % 256) return set_error(FEH_EINVAL, "workspace must be 256-byte aligned");
        const int C = ne * D * D;
        FRun R{p, p, kind, ne, C, Lo, static_cast<char *>(work_dev)};
        R.fp.L = p.L * C;
        R.fp.prof_on = false;
        if ((double)(p.N / p.n[D - 1]) * R.fp.L >= 2147483647.0)
            return set_error(FEH_ENOTSUP, "grid too large for the finite-strain solver");
        FsParams prm{n_steps, max_newton, max_cg, newton_tol, equil_tol, cg_tol};
        FsOut out;
        int rc;
        if (p.prec == FEH_FP64)
            rc = D == 3 ? fs_solve_t<double, 3>(R, Fbar_host, prm, F_dev, P_dev, out)
                        : fs_solve_t<double, 2>(R, Fbar_host, prm, F_dev, P_dev, out);
        else
            rc = D == 3 ? fs_solve_t<float, 3>(R, Fbar_host, prm, F_dev, P_dev, out)
                        : fs_solve_t<float, 2>(R, Fbar_host, prm, F_dev, P_dev, out);
        CK(rc);
        if (P_mean_host) std::memcpy(P_mean_host, out.pmean.data(), out.pmean.size() * sizeof(double));
        rc = FEH_OK;
        for (int l = 0; l < p.L; ++l) {
            if (report_host) {
                report_host[l].newton_iterations = out.newton[l];
                report_host[l].cg_iterations = out.cg[l];
                report_host[l].status = out.status[l];
                report_host[l].pad = 0;
                report_host[l].rel_equilibrium = out.rel_eq[l];
                report_host[l].rel_increment = out.rel_inc[l];
            }
            if (out.status[l] != FEH_OK) rc = FEH_ENOCONV;
        }
        if (rc == FEH_ENOCONV) return set_error(rc, "Newton did not converge within max_newton");
        return FEH_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FEH_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(FEH_EINVAL, "unexpected host exception");
    }
}

}  // extern "C"
