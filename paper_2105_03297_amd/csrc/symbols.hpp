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
constexpr int kVecBlocks = 512;  // blocks per load case of the vector kernels
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
    double g[6][4][3];   // FE: shape-function gradients per element and vertex (physical units)
    double h[3];
    int n[3];
    int nh;              // half-spectrum length of the last axis
    double tiny;         // symbols with sum |D|^2 <= tiny are projected out
};

// Shape-function gradients of a simplex with vertices X[0..dim] (physical
// units): barycentric coordinate c >= 1 is row c - 1 of J^-1 (x - X0) with
// J = [X1 - X0, ..., Xd - X0]; coordinate 0 is one minus the others.
void simplex_gradients(int dim, const double (*X)[3], double (*g)[3]) {
    double J[3][3] = {}, Ji[3][3] = {};
    for (int c = 1; c <= dim; ++c)
        for (int a = 0; a < dim; ++a) J[a][c - 1] = X[c][a] - X[0][a];
    if (dim == 2) {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
    } else {
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        // (J^-1)_ij = cofactor of J_ji / det (cyclic index form)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
                Ji[i][j] = (J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1]) / det;
            }
    }
    for (int a = 0; a < dim; ++a) {
        double s = 0.0;
        for (int c = 1; c <= dim; ++c) {
            g[c][a] = Ji[c - 1][a];
            s += g[c][a];
        }
        g[0][a] = -s;
    }
}

// Element vertex offsets (voxel units): 2D triangles (00, 10, 01) and
// (11, 01, 10); 3D Kuhn tetrahedra 0, e_a, e_a + e_b, (1,1,1) along the axis
// paths (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x).
void element_offsets(int dim, int e, int (*r)[3]) {
    std::memset(r, 0, sizeof(int) * 4 * 3);
    if (dim == 2) {
        static const int T[2][3][2] = {{{0, 0}, {1, 0}, {0, 1}}, {{1, 1}, {0, 1}, {1, 0}}};
        for (int c = 0; c < 3; ++c) {
            r[c][0] = T[e][c][0];
            r[c][1] = T[e][c][1];
        }
        return;
    }
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int c = 1; c <= 3; ++c) {
        for (int a = 0; a < 3; ++a) r[c][a] = r[c - 1][a];
        r[c][P[e][c - 1]] += 1;
    }
}

// FE: vertex offset of (element, vertex) as bits (bit a: +1 voxel along axis
// a), constants so that the phase lookup below resolves at compile time.
__host__ __device__ constexpr int fe_corner(int dim, int e, int c) {
    constexpr int c2[2][3] = {{0, 1, 2}, {3, 2, 1}};
    constexpr int c3[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
    return dim == 2 ? c2[e][c] : c3[e][c];
}

SymArgs make_sym_args(const feh_plan &p, int kind) {
    SymArgs s{};
    for (int a = 0; a < 3; ++a) {
        s.h[a] = p.h[a];
        s.n[a] = (int)p.n[a];
    }
    s.nh = (int)p.nh;
    double sc = 0.0;
    for (int a = 0; a < p.dim; ++a) sc += 1.0 / (p.h[a] * p.h[a]);
    s.tiny = 1e-24 * sc;
    if (kind == K_FE) {
        for (int e = 0; e < points_of(K_FE, p.dim); ++e) {
            int R[4][3];
            element_offsets(p.dim, e, R);
            double X[4][3] = {};
            for (int c = 0; c <= p.dim; ++c) {
                for (int a = 0; a < p.dim; ++a) X[c][a] = R[c][a] * p.h[a];
            }
            simplex_gradients(p.dim, X, s.g[e]);
        }
    }
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
        C64 P[1 << DIM];
        #pragma unroll
        for (int r = 0; r < (1 << DIM); ++r) {
            C64 v{1.0, 0.0};
            #pragma unroll
            for (int a = 0; a < DIM; ++a)
                if (r & (1 << a)) v = cmul(v, C64{cs[a], sn[a]});
            P[r] = v;
        }
        #pragma unroll
        for (int e = 0; e < NE; ++e)
            #pragma unroll
            for (int a = 0; a < DIM; ++a) {
                C64 v{0.0, 0.0};
                #pragma unroll
                for (int c = 0; c <= DIM; ++c) {
                    const C64 ph = P[fe_corner(DIM, e, c)];
                    v = cadd(v, cscale(ph, sa.g[e][c][a]));
                }
                D[e][a] = v;
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

// Inverse of M = 1/2 (I + sum_T D_T D_T^H) (normalised symbol), by cofactors.
template <int DIM, int NE>
__device__ __forceinline__ void metric_inverse(const C64 (&D)[NE][DIM], C64 (&Mi)[DIM][DIM]) {
    C64 M[DIM][DIM];
    #pragma unroll
    for (int x = 0; x < DIM; ++x)
        #pragma unroll
        for (int y = 0; y < DIM; ++y) {
            C64 s{x == y ? 1.0 : 0.0, 0.0};
            #pragma unroll
            for (int e = 0; e < NE; ++e) s = cadd(s, cmulc(D[e][x], D[e][y]));
            M[x][y] = cscale(s, 0.5);
        }
    if constexpr (DIM == 2) {
        const C64 det = csub(cmul(M[0][0], M[1][1]), cmul(M[0][1], M[1][0]));
        const double dn = 1.0 / (det.x * det.x + det.y * det.y);
        const C64 id = {det.x * dn, -det.y * dn};
        Mi[0][0] = cmul(M[1][1], id);
        Mi[1][1] = cmul(M[0][0], id);
        Mi[0][1] = cmul(C64{-M[0][1].x, -M[0][1].y}, id);
        Mi[1][0] = cmul(C64{-M[1][0].x, -M[1][0].y}, id);
    } else {
        C64 cof[3][3];
        #pragma unroll
        for (int i = 0; i < 3; ++i)
            #pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int r1 = (i + 1) % 3, r2 = (i + 2) % 3, c1 = (j + 1) % 3, c2 = (j + 2) % 3;
                cof[i][j] = csub(cmul(M[r1][c1], M[r2][c2]), cmul(M[r1][c2], M[r2][c1]));
            }
        const C64 det = cadd(cadd(cmul(M[0][0], cof[0][0]), cmul(M[0][1], cof[0][1])), cmul(M[0][2], cof[0][2]));
        const double dn = 1.0 / (det.x * det.x + det.y * det.y);
        const C64 id = {det.x * dn, -det.y * dn};
        #pragma unroll
        for (int i = 0; i < 3; ++i)
            #pragma unroll
            for (int j = 0; j < 3; ++j) Mi[i][j] = cmul(cof[j][i], id);
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
