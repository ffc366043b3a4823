// Discrete derivative symbols of the strain-space solvers (small and finite
// strain): the derivative kinds of Sec. "Discrete projection", their Fourier
// symbols D_T(k) per evaluation point T evaluated on the fly from the
// wavevector index, and the small D x D Hermitian inverse of the small-strain
// projection.  Shared by spectral.hip and finite.hip (internal linkage).
#pragma once

#include <cmath>
#include <cstring>

#include "device_common.hpp"

namespace feh {
namespace {

constexpr int kThreads = 256;
constexpr int kVecBlocks = 2048;  // blocks per load case of the vector kernels
constexpr int kPostBlocks = 256;

enum Kind { K_FE = FEH_DERIV_FE, K_FD = FEH_DERIV_FD, K_CD = FEH_DERIV_CD, K_LS = FEH_DERIV_LS,
            K_FOURIER = FEH_DERIV_FOURIER, K_FOURIER2 = FEH_DERIV_FOURIER2 };

int points_of(int kind, int dim) {
    if (dim != 2 && dim != 3) return -1;
    switch (kind) {
    case K_FE: return dim == 3 ? 6 : 2;
    case K_FOURIER2: return dim == 2 ? 2 : -1;
    case K_LS: return dim == 2 ? 1 : -1;
    case K_FD:
    case K_CD:
    case K_FOURIER: return 1;
    default: return -1;
    }
}

constexpr int nsym(int dim) { return dim == 3 ? 6 : 3; }

// Symbol description passed by value to the projection kernel.
struct SymArgs {
    double h[3];
    int n[3];
    int nh;              // half-spectrum length of the last axis
    double tiny;         // symbols with sum |D|^2 <= tiny are projected out
};

SymArgs make_sym_args(const feh_plan &p, int) {
    SymArgs s{};
    for (int a = 0; a < 3; ++a) {
        s.h[a] = p.h[a];
        s.n[a] = (int)p.n[a];
    }
    s.nh = (int)p.nh;
    double sc = 0.0;
    for (int a = 0; a < p.dim; ++a) sc += 1.0 / (p.h[a] * p.h[a]);
    s.tiny = 1e-24 * sc;
    return s;
}

// ---------------------------------------------------------------------------
// device: symbols
// ---------------------------------------------------------------------------
using C64 = Cx<double>;

template <int DIM, int KIND>
struct Pts {
    static constexpr int NE = KIND == K_FE ? (DIM == 3 ? 6 : 2) : (KIND == K_FOURIER2 ? 2 : 1);
};

// Symbol D[T][a] at half-spectrum index k, normalised to sum |D|^2 = 1.
// FLIP evaluates the Fourier derivatives with +pi/h instead of -pi/h at
// Nyquist indices (the mirror image needed for the Hermitian part).  Returns
// false where the mode is projected out; nyq reports a Nyquist component.
template <int DIM, int KIND, bool FLIP>
__device__ __forceinline__ bool symbol_at(const SymArgs &sa, long long k, C64 (&D)[Pts<DIM, KIND>::NE][DIM],
                                          bool &nyq) {
    constexpr int NE = Pts<DIM, KIND>::NE;
    int idx[3];
    long long rest = k;
    idx[DIM - 1] = (int)(rest % sa.nh);
    rest /= sa.nh;
    if (DIM == 3) {
        idx[1] = (int)(rest % sa.n[1]);
        rest /= sa.n[1];
    }
    idx[0] = (int)rest;
    double th[DIM], cs[DIM], sn[DIM];
    nyq = false;
    #pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int n = sa.n[a];
        int m = idx[a];
        if (2 * m >= n) m -= n;  // range [-n/2, n/2 - 1] (even n) or [-(n-1)/2, (n-1)/2] (odd n)
        const bool ny = 2 * m == -n;
        nyq = nyq || ny;
        if (FLIP && ny) m = -m;
        const double x = 2.0 * (double)m / (double)n;  // theta / pi
        th[a] = M_PI * x;
        sincospi(x, &sn[a], &cs[a]);
    }
    if constexpr (KIND == K_FE) {
        // vertex phases e^{i k.r} of the voxel corners (bit a: +1 along axis a)
        C64 P[1 << DIM];
        #pragma unroll
        for (int r = 0; r < (1 << DIM); ++r) {
            C64 v{1.0, 0.0};
            #pragma unroll
            for (int a = 0; a < DIM; ++a)
                if (r & (1 << a)) v = cmul(v, C64{cs[a], sn[a]});
            P[r] = v;
        }
        // the gradient of a linear simplex along a voxel edge of its vertex
        // path is the difference of the edge's end values over h_a: tetrahedron
        // (A0, A1, A2) runs 0 -> e_A0 -> e_A0 + e_A1 -> (1,1,1); triangle 0 has
        // edges 00-10 (x) and 00-01 (y), triangle 1 edges 01-11 (x) and 10-11 (y)
        double ih[DIM];
        #pragma unroll
        for (int a = 0; a < DIM; ++a) ih[a] = 1.0 / sa.h[a];
        if constexpr (DIM == 3) {
            constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
            #pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int A0 = perm[e][0], A1 = perm[e][1], A2 = perm[e][2];
                const int V1 = 1 << A0, V2 = V1 | (1 << A1);
                D[e][A0] = cscale(csub(P[V1], P[0]), ih[A0]);
                D[e][A1] = cscale(csub(P[V2], P[V1]), ih[A1]);
                D[e][A2] = cscale(csub(P[7], P[V2]), ih[A2]);
            }
        } else {
            D[0][0] = cscale(csub(P[1], P[0]), ih[0]);
            D[0][1] = cscale(csub(P[2], P[0]), ih[1]);
            D[1][0] = cscale(csub(P[3], P[2]), ih[0]);
            D[1][1] = cscale(csub(P[3], P[1]), ih[1]);
        }
    } else if constexpr (KIND == K_FD) {
        #pragma unroll
        for (int a = 0; a < DIM; ++a) D[0][a] = C64{(cs[a] - 1.0) / sa.h[a], sn[a] / sa.h[a]};
    } else if constexpr (KIND == K_CD) {
        #pragma unroll
        for (int a = 0; a < DIM; ++a) D[0][a] = C64{0.0, sn[a] / sa.h[a]};
    } else if constexpr (KIND == K_LS) {
        const C64 e0m = {cs[0] - 1.0, sn[0]}, e1m = {cs[1] - 1.0, sn[1]};
        const C64 e0p = {cs[0] + 1.0, sn[0]}, e1p = {cs[1] + 1.0, sn[1]};
        D[0][0] = cscale(cmul(e0m, e1p), 0.5 / sa.h[0]);
        D[0][1] = cscale(cmul(e0p, e1m), 0.5 / sa.h[1]);
    } else if constexpr (KIND == K_FOURIER) {
        #pragma unroll
        for (int a = 0; a < DIM; ++a) D[0][a] = C64{0.0, th[a] / sa.h[a]};
    } else {  // two-point Fourier: i k e^{-i s} and i k e^{+i s}, s = (theta_0 + theta_1) / 6
        double ss, cc;
        sincos((th[0] + th[1]) / 6.0, &ss, &cc);
        #pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double ka = th[a] / sa.h[a];
            D[0][a] = C64{ka * ss, ka * cc};   // i k (cos s - i sin s)
            D[1][a] = C64{-ka * ss, ka * cc};  // i k (cos s + i sin s)
        }
    }
    double S = 0.0;
    #pragma unroll
    for (int e = 0; e < NE; ++e)
        #pragma unroll
        for (int a = 0; a < DIM; ++a) S += D[e][a].x * D[e][a].x + D[e][a].y * D[e][a].y;
    if (!(S > sa.tiny)) return false;
    const double is = 1.0 / sqrt(S);
    #pragma unroll
    for (int e = 0; e < NE; ++e)
        #pragma unroll
        for (int a = 0; a < DIM; ++a) D[e][a] = cscale(D[e][a], is);
    return true;
}

// Inverse of the Hermitian M = 1/2 (I + sum_T D_T D_T^H) (normalised symbol)
// by the adjugate: real diagonal Id and upper triangle Io = (01, 02, 12)
// (2D: Io[0] = 01).
template <int DIM, int NE>
__device__ __forceinline__ void metric_inverse(const C64 (&D)[NE][DIM], double (&Id)[DIM], C64 (&Io)[3]) {
    double d[DIM];
    C64 o[3] = {C64{0.0, 0.0}, C64{0.0, 0.0}, C64{0.0, 0.0}};
    #pragma unroll
    for (int x = 0; x < DIM; ++x) {
        double s = 1.0;
        #pragma unroll
        for (int e = 0; e < NE; ++e) s += D[e][x].x * D[e][x].x + D[e][x].y * D[e][x].y;
        d[x] = 0.5 * s;
    }
    #pragma unroll
    for (int u = 0; u < (DIM == 3 ? 3 : 1); ++u) {
        const int x = (DIM == 3 && u == 2) ? 1 : 0, y = (DIM == 3 && u >= 1) ? 2 : 1;
        C64 s{0.0, 0.0};
        #pragma unroll
        for (int e = 0; e < NE; ++e) s = cadd(s, cmulc(D[e][x], D[e][y]));
        o[u] = cscale(s, 0.5);
    }
    if constexpr (DIM == 2) {
        const double id = 1.0 / (d[0] * d[1] - (o[0].x * o[0].x + o[0].y * o[0].y));
        Id[0] = d[1] * id;
        Id[1] = d[0] * id;
        Io[0] = cscale(o[0], -id);
        Io[1] = Io[2] = C64{0.0, 0.0};
    } else {
        const C64 a = o[0], b = o[1], c = o[2];
        const double C0 = d[1] * d[2] - (c.x * c.x + c.y * c.y);
        const double C1 = d[0] * d[2] - (b.x * b.x + b.y * b.y);
        const double C2 = d[0] * d[1] - (a.x * a.x + a.y * a.y);
        const C64 A01 = csub(cmulc(b, c), cscale(a, d[2]));  // b conj(c) - a d2
        const C64 A02 = csub(cmul(a, c), cscale(b, d[1]));   // a c - b d1
        const C64 A12 = csub(cmulc(b, a), cscale(c, d[0]));  // b conj(a) - c d0
        const double det = d[0] * C0 + (a.x * A01.x + a.y * A01.y) + (b.x * A02.x + b.y * A02.y);
        const double id = 1.0 / det;
        Id[0] = C0 * id;
        Id[1] = C1 * id;
        Id[2] = C2 * id;
        Io[0] = cscale(A01, id);
        Io[1] = cscale(A02, id);
        Io[2] = cscale(A12, id);
    }
}

// component index of tensor entry (i, j) in the symmetric storage
template <int DIM>
__host__ __device__ constexpr int sidx(int i, int j) {
    return i == j ? i : (DIM == 2 ? 2 : (i + j == 3 ? 3 : (i + j == 2 ? 4 : 5)));
}

int grid_of(long long n) {
    long long g = (n + kThreads - 1) / kThreads;
    if (g > 8192) g = 8192;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace
}  // namespace feh
