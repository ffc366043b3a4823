// Post-processing of converged displacement fluctuations.
//
// Per element: e = Ebar + sym(grad u) (small-strain appendix), sigma = C e;
// volume averages <sigma>_l and the energy matrix W_lm = <e_l : C : e_m>
// (all elements carry the same volume, so the averages are plain means).
// W is the Hill energy form of the effective stiffness, second order in the
// CG error.  One grid axis enumerates the scalar quantities (stress means of
// each load case, and each load-case pair of W); partial sums per block are
// combined in a fixed order by k_reduce_slots.
#include <algorithm>

#include "device_common.hpp"

namespace feh {
namespace {

constexpr int kThreads = 256;

// symmetric strain of every element of a voxel from its corner
// displacements; e[t] = (xx, yy, zz, yz, xz, xy) (tensor components)
template <typename T>
__device__ __forceinline__ void strains3(const T (&P)[8][3], const T (&ih)[3], double (&e)[6][6]) {
    constexpr int KP[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    #pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int a0 = KP[t][0], a1 = KP[t][1], a2 = KP[t][2];
        const int v1 = 1 << a0, v2 = v1 | (1 << a1);
        double G[3][3];
        #pragma unroll
        for (int i = 0; i < 3; ++i) {
            G[i][a0] = double(P[v1][i] - P[0][i]) * double(ih[a0]);
            G[i][a1] = double(P[v2][i] - P[v1][i]) * double(ih[a1]);
            G[i][a2] = double(P[7][i] - P[v2][i]) * double(ih[a2]);
        }
        e[t][0] = G[0][0];
        e[t][1] = G[1][1];
        e[t][2] = G[2][2];
        e[t][3] = 0.5 * (G[1][2] + G[2][1]);
        e[t][4] = 0.5 * (G[0][2] + G[2][0]);
        e[t][5] = 0.5 * (G[0][1] + G[1][0]);
    }
}

// 2D: element 0 nodes 00,10,01; element 1 nodes 11,01,10; e[t] = (xx, yy, xy)
template <typename T>
__device__ __forceinline__ void strains2(const T (&P)[4][2], const T (&ih)[3], double (&e)[2][3]) {
    const double hx = ih[0], hy = ih[1];
    double G[2][2];
    G[0][0] = double(P[1][0] - P[0][0]) * hx;
    G[0][1] = double(P[2][0] - P[0][0]) * hy;
    G[1][0] = double(P[1][1] - P[0][1]) * hx;
    G[1][1] = double(P[2][1] - P[0][1]) * hy;
    e[0][0] = G[0][0];
    e[0][1] = G[1][1];
    e[0][2] = 0.5 * (G[0][1] + G[1][0]);
    G[0][0] = double(P[3][0] - P[2][0]) * hx;
    G[0][1] = double(P[3][0] - P[1][0]) * hy;
    G[1][0] = double(P[3][1] - P[2][1]) * hx;
    G[1][1] = double(P[3][1] - P[1][1]) * hy;
    e[1][0] = G[0][0];
    e[1][1] = G[1][1];
    e[1][2] = 0.5 * (G[0][1] + G[1][0]);
}

template <typename T>
struct PK {
    const T *u;         // SoA [L][D][N], may be null (zero fluctuation)
    const double *Ebar; // [L][D][D]
    const T *lam;
    const T *mu;
    T *strain;          // [L][N][ne][D][D] or null
    T *stress;
    double *partial;    // [slot][nblk]
    int n0, n1, n2;     // 2D: n1 = 1, n2 = n[1]
    long long N;
    int L, nblk, nsym;
    int G, nbatch;      // load cases per microstructure, microstructures
    T ih[3];
    int grad_only;      // projection test: write sym(grad u) only (no Ebar, no sums)
};

// Node offsets of the corners of voxel v (corner c = c0 + 2 c1 (+ 4 c2)),
// periodic.  Voxel indices fit 32 bits (N <= 2^31), so the coordinates come
// from 32-bit divisions; the offsets serve every load case of the voxel.
template <int DIM>
__device__ __forceinline__ void corner_offsets(int n0, int n1, int n2, long long v, uint32_t (&idx)[1 << DIM]) {
    const uint32_t vv = (uint32_t)v;
    const uint32_t r = vv / (uint32_t)n2;
    const int k2 = (int)(vv - r * (uint32_t)n2);
    const int k1 = (int)(r % (uint32_t)n1);
    const int k0 = (int)(r / (uint32_t)n1);
    const int j0 = k0 + 1 == n0 ? 0 : k0 + 1, j1 = k1 + 1 == n1 ? 0 : k1 + 1, j2 = k2 + 1 == n2 ? 0 : k2 + 1;
    #pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        int i0, i1, i2;
        if (DIM == 3) {
            i0 = (c & 1) ? j0 : k0;
            i1 = ((c >> 1) & 1) ? j1 : k1;
            i2 = ((c >> 2) & 1) ? j2 : k2;
        } else {
            i0 = (c & 1) ? j0 : k0;
            i1 = 0;
            i2 = ((c >> 1) & 1) ? j2 : k2;
        }
        idx[c] = ((uint32_t)i0 * (uint32_t)n1 + (uint32_t)i1) * (uint32_t)n2 + (uint32_t)i2;
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void load_corners(const PK<T> &a, int l, const uint32_t (&idx)[1 << DIM],
                                             T (&P)[1 << DIM][DIM]) {
    const T *ub = a.u + (long long)l * DIM * a.N;
    #pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        #pragma unroll
        for (int i = 0; i < DIM; ++i) P[c][i] = a.u ? ub[i * a.N + idx[c]] : T(0);
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void voxel_strains(const PK<T> &a, int l, const uint32_t (&cidx)[1 << DIM], bool add_ebar,
                                              double (&e)[DIM == 3 ? 6 : 2][DIM == 3 ? 6 : 3]) {
    T P[1 << DIM][DIM];
    load_corners<T, DIM>(a, l, cidx, P);
    if constexpr (DIM == 3) {
        strains3<T>(P, a.ih, e);
        if (add_ebar) {
            const double *E = a.Ebar + l * 9;
            const double eb[6] = {E[0], E[4], E[8], E[5], E[2], E[1]};
            #pragma unroll
            for (int t = 0; t < 6; ++t)
                #pragma unroll
                for (int k = 0; k < 6; ++k) e[t][k] += eb[k];
        }
    } else {
        strains2<T>(P, a.ih, e);
        if (add_ebar) {
            const double *E = a.Ebar + l * 4;
            const double eb[3] = {E[0], E[3], E[1]};
            #pragma unroll
            for (int t = 0; t < 2; ++t)
                #pragma unroll
                for (int k = 0; k < 3; ++k) e[t][k] += eb[k];
        }
    }
}

// sigma (symmetric components) from a strain in the same storage
template <int DIM>
__device__ __forceinline__ void stress_of(const double *e, double lam, double mu, double *s) {
    if constexpr (DIM == 3) {
        const double lt = lam * (e[0] + e[1] + e[2]);
        s[0] = lt + 2 * mu * e[0];
        s[1] = lt + 2 * mu * e[1];
        s[2] = lt + 2 * mu * e[2];
        s[3] = 2 * mu * e[3];
        s[4] = 2 * mu * e[4];
        s[5] = 2 * mu * e[5];
    } else {
        const double lt = lam * (e[0] + e[1]);
        s[0] = lt + 2 * mu * e[0];
        s[1] = lt + 2 * mu * e[1];
        s[2] = 2 * mu * e[2];
    }
}

template <int DIM>
__device__ __forceinline__ double ddot(const double *e, const double *s) {
    if constexpr (DIM == 3) return e[0] * s[0] + e[1] * s[1] + e[2] * s[2] + 2.0 * (e[3] * s[3] + e[4] * s[4] + e[5] * s[5]);
    else return e[0] * s[0] + e[1] * s[1] + 2.0 * e[2] * s[2];
}

// write a symmetric tensor as a full D x D block
template <typename T, int DIM>
__device__ __forceinline__ void put_full(T *dst, const double *s) {
    if constexpr (DIM == 3) {
        dst[0] = T(s[0]); dst[1] = T(s[5]); dst[2] = T(s[4]);
        dst[3] = T(s[5]); dst[4] = T(s[1]); dst[5] = T(s[3]);
        dst[6] = T(s[4]); dst[7] = T(s[3]); dst[8] = T(s[2]);
    } else {
        dst[0] = T(s[0]); dst[1] = T(s[2]);
        dst[2] = T(s[2]); dst[3] = T(s[1]);
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_post(PK<T> a) {
    constexpr int NE = DIM == 3 ? 6 : 2;
    constexpr int NS = DIM == 3 ? 6 : 3;
    __shared__ double red[kThreads / 64];
    const int qslot = blockIdx.y;  // quantity
    const int blk = blockIdx.x;
    double acc[NS];
    #pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    int l = qslot, m = -1;
    if (qslot >= a.L) {
        // pair index -> microstructure b and (l, m), l <= m, both in its group
        int rem = qslot - a.L;
        const int npg = a.G * (a.G + 1) / 2;
        const int b = rem / npg;
        rem -= b * npg;
        int li = 0;
        while (rem >= a.G - li) {
            rem -= a.G - li;
            ++li;
        }
        l = b * a.G + li;
        m = l + rem;
    }
    const long long mo = (long long)(l / a.G) * a.N;
    for (long long v = blk * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)a.nblk * kThreads) {
        const double lam = double(a.lam[mo + v]), mu = double(a.mu[mo + v]);
        uint32_t cidx[1 << DIM];
        corner_offsets<DIM>(a.n0, a.n1, a.n2, v, cidx);
        double e[NE][NS];
        voxel_strains<T, DIM>(a, l, cidx, true, e);
        if (m < 0) {
            #pragma unroll
            for (int t = 0; t < NE; ++t) {
                double s[NS];
                stress_of<DIM>(e[t], lam, mu, s);
                #pragma unroll
                for (int k = 0; k < NS; ++k) acc[k] += s[k];
                const long long off = (((long long)l * a.N + v) * NE + t) * DIM * DIM;
                if (a.strain) put_full<T, DIM>(a.strain + off, e[t]);
                if (a.stress) put_full<T, DIM>(a.stress + off, s);
            }
        } else {
            double f[NE][NS];
            voxel_strains<T, DIM>(a, m, cidx, true, f);
            #pragma unroll
            for (int t = 0; t < NE; ++t) {
                double s[NS];
                stress_of<DIM>(f[t], lam, mu, s);
                acc[0] += ddot<DIM>(e[t], s);
            }
        }
    }
    const int nout = (m < 0) ? NS : 1;
    for (int k = 0; k < nout; ++k) {
        const double s = block_sum<kThreads>(acc[k], red);
        if (threadIdx.x == 0) {
            const long long slot = (m < 0) ? (long long)l * NS + k : (long long)a.L * NS + (qslot - a.L);
            a.partial[slot * a.nblk + blk] = s;
        }
    }
}

template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_grad(PK<T> a) {
    constexpr int NE = DIM == 3 ? 6 : 2;
    constexpr int NS = DIM == 3 ? 6 : 3;
    const int l = blockIdx.y;
    for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)gridDim.x * kThreads) {
        double e[NE][NS];
        uint32_t cidx[1 << DIM];
        corner_offsets<DIM>(a.n0, a.n1, a.n2, v, cidx);
        voxel_strains<T, DIM>(a, l, cidx, false, e);
        #pragma unroll
        for (int t = 0; t < NE; ++t) put_full<T, DIM>(a.strain + (((long long)l * a.N + v) * NE + t) * DIM * DIM, e[t]);
    }
}

// Sensitivities of sum_lm w_lm W_lm to the per-voxel Lame constants.  W_lm is
// stationary in the fluctuations (energy minimum of the weak form), so only
// the explicit dependence on C counts:
//   g_lam[v] = sum_pairs w <tr e_l tr e_m>_v,  g_mu[v] = sum_pairs w <2 e_l : e_m>_v,
// <.>_v the element terms of voxel v with the weights of the cell average
// (scale = 1 / (N n_e)).  The pair list holds l <= m within one
// microstructure, grouped by microstructure (pairs gofs[b] .. gofs[b+1] - 1
// write field b); an off-diagonal pair's weight already carries w_lm + w_ml.
// g_E non-null: one field g_E = aE g_lam + bE g_mu (the Young's modulus
// sensitivity through the Lame maps at a uniform nu) instead of the two.
template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_sens(PK<T> a, const int *pl, const int *pm, const double *pw,
                                                   const int *gofs, double scale, T *g_lam, T *g_mu, T *g_E,
                                                   double aE, double bE) {
    constexpr int NE = DIM == 3 ? 6 : 2;
    constexpr int NS = DIM == 3 ? 6 : 3;
    for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < a.N; v += (long long)gridDim.x * kThreads) {
      uint32_t cidx[1 << DIM];
      corner_offsets<DIM>(a.n0, a.n1, a.n2, v, cidx);
      for (int bb = 0; bb < a.nbatch; ++bb) {
        double gl = 0.0, gm = 0.0;
        for (int q = gofs[bb]; q < gofs[bb + 1]; ++q) {
            const int l = pl[q], m = pm[q];
            const double w = pw[q];
            double e[NE][NS], f[NE][NS];
            voxel_strains<T, DIM>(a, l, cidx, true, e);
            if (m != l) {
                voxel_strains<T, DIM>(a, m, cidx, true, f);
            } else {
                #pragma unroll
                for (int t = 0; t < NE; ++t)
                    #pragma unroll
                    for (int k = 0; k < NS; ++k) f[t][k] = e[t][k];
            }
            double sl = 0.0, sm = 0.0;
            #pragma unroll
            for (int t = 0; t < NE; ++t) {
                double te, tf, dd;
                if constexpr (DIM == 3) {
                    te = e[t][0] + e[t][1] + e[t][2];
                    tf = f[t][0] + f[t][1] + f[t][2];
                    dd = e[t][0] * f[t][0] + e[t][1] * f[t][1] + e[t][2] * f[t][2] +
                         2.0 * (e[t][3] * f[t][3] + e[t][4] * f[t][4] + e[t][5] * f[t][5]);
                } else {
                    te = e[t][0] + e[t][1];
                    tf = f[t][0] + f[t][1];
                    dd = e[t][0] * f[t][0] + e[t][1] * f[t][1] + 2.0 * e[t][2] * f[t][2];
                }
                sl += te * tf;
                sm += 2.0 * dd;
            }
            gl += w * sl;
            gm += w * sm;
        }
        if (g_E) {
            g_E[(long long)bb * a.N + v] = T((aE * gl + bE * gm) * scale);
        } else {
            g_lam[(long long)bb * a.N + v] = T(gl * scale);
            g_mu[(long long)bb * a.N + v] = T(gm * scale);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Plane-marching variants (microstructures of at most kMarchG load cases):
// a workgroup of VY x VZ voxels (3D 8 x 32, 2D one row of 256) marches
// along axis 0 over a chunk of kMarchChunk planes, each thread reading the
// corner nodes of its voxel column straight from memory.  Consecutive
// workgroups (the same XCD after xcd_remap) cover the load cases of one tile
// and neighbouring tiles, so a node plane is fetched from HBM about once and
// served from L2 to the other corners, quantities and load cases that use it.
// ---------------------------------------------------------------------------
constexpr int kMarchG = 6;
constexpr int kMarchChunk = 16;

template <int DIM>
struct MTile;
template <>
struct MTile<3> {
    static constexpr int VY = 8, VZ = 32;
};
template <>
struct MTile<2> {
    static constexpr int VY = 1, VZ = 256;
};

struct MarchGeom {
    int nty, ntz, nchunk;
};

template <int DIM>
MarchGeom march_geom(const feh_plan &p) {
    using TL = MTile<DIM>;
    const int n0 = (int)p.n[0], n1 = DIM == 3 ? (int)p.n[1] : 1, n2 = (int)p.n[DIM - 1];
    return MarchGeom{(n1 + TL::VY - 1) / TL::VY, (n2 + TL::VZ - 1) / TL::VZ, (n0 + kMarchChunk - 1) / kMarchChunk};
}

// In-plane offsets of the corner nodes of a voxel column (corner
// c = cx + 2 cy (+ 4 cz) with cx the axis-0 bit, periodic).
template <int DIM>
struct ColumnCorners {
    uint32_t o[4];  // in-plane offsets of the corners (cy, cz) = 00, 10, 01, 11 (3D); 2D cz = 0, 1
    __device__ __forceinline__ void init(int n1, int n2, int y, int z) {
        const int z1 = z + 1 == n2 ? 0 : z + 1;
        if constexpr (DIM == 3) {
            const int y1 = y + 1 == n1 ? 0 : y + 1;
            o[0] = (uint32_t)y * n2 + z;
            o[1] = (uint32_t)y1 * n2 + z;
            o[2] = (uint32_t)y * n2 + z1;
            o[3] = (uint32_t)y1 * n2 + z1;
        } else {
            o[0] = (uint32_t)z;
            o[1] = (uint32_t)z1;
            o[2] = o[3] = 0;
        }
    }
};

// Corner values of load case l of the voxel between node planes at offsets
// xa (cx = 0) and xb (cx = 1).
template <typename T, int DIM>
__device__ __forceinline__ void column_corners(const PK<T> &a, int l, uint32_t xa, uint32_t xb,
                                               const ColumnCorners<DIM> &cc, T (&P)[1 << DIM][DIM]) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i) {
        const T *ui = a.u + ((long long)l * DIM + i) * a.N;
        #pragma unroll
        for (int c = 0; c < (1 << DIM); ++c) P[c][i] = ui[((c & 1) ? xb : xa) + cc.o[c >> 1]];
    }
}

template <typename T, int DIM>
__device__ __forceinline__ void for_corners_zero(T (&P)[1 << DIM][DIM]) {
    #pragma unroll
    for (int c = 0; c < (1 << DIM); ++c)
        #pragma unroll
        for (int i = 0; i < DIM; ++i) P[c][i] = T(0);
}

// Displacement gradient of element TT of the voxel plus Ebar (full D x D,
// g[i][a] = d u_i / d x_a + Ebar_ia), one FMA per entry: the element's edge
// along axis a starts at corner BASE[TT][a] (3D: tetrahedron with axis path
// (a0, a1, a2) walks corners 0, 1<<a0, 1<<a0 | 1<<a1, 7; 2D: triangle 0 is
// nodes 00, 10, 01, triangle 1 nodes 11, 01, 10).  The symmetric part of g is
// the element strain e; the unrolled callers share the twelve (3D) edge
// differences between elements.
template <typename R, typename T, int DIM, int TT>
__device__ __forceinline__ void element_grad(const T (&P)[1 << DIM][DIM], const T (&ih)[3], const R (&Eb)[DIM][DIM],
                                             R (&g)[DIM][DIM]) {
    constexpr int BASE3[6][3] = {{0, 1, 3}, {0, 5, 1}, {2, 0, 3}, {6, 0, 2}, {4, 5, 0}, {6, 4, 0}};
    constexpr int BASE2[2][2] = {{0, 0}, {2, 1}};
    #pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        const int c0 = DIM == 3 ? BASE3[TT][ax] : BASE2[TT][ax];
        const int c1 = c0 | (1 << ax);  // corner bit of axis ax: 3D c = cx + 2 cy + 4 cz, 2D c = cx + 2 cz
        #pragma unroll
        for (int i = 0; i < DIM; ++i) g[i][ax] = fma(R(P[c1][i] - P[c0][i]), R(ih[ax]), Eb[i][ax]);
    }
}

template <int DIM, typename R>
__device__ __forceinline__ void ebar_full(const double *Ebar, int l, R (&Eb)[DIM][DIM]) {
    #pragma unroll
    for (int i = 0; i < DIM; ++i)
        #pragma unroll
        for (int j = 0; j < DIM; ++j) Eb[i][j] = R(Ebar[(l * DIM + i) * DIM + j]);
}

// Sums over the voxel's elements of (tr e)^2 and e : e for corner values P,
// in arithmetic R.
template <typename R, typename T, int DIM, int TT = 0>
__device__ __forceinline__ void self_sums(const T (&P)[1 << DIM][DIM], const T (&ih)[3], const R (&Eb)[DIM][DIM], R &st,
                                          R &se) {
    constexpr int NEL = DIM == 3 ? 6 : 2;
    if constexpr (TT < NEL) {
        R g[DIM][DIM];
        element_grad<R, T, DIM, TT>(P, ih, Eb, g);
        R tr = g[0][0], dg = g[0][0] * g[0][0], off = R(0);
        #pragma unroll
        for (int i = 1; i < DIM; ++i) {
            tr += g[i][i];
            dg = fma(g[i][i], g[i][i], dg);
        }
        #pragma unroll
        for (int i = 0; i < DIM; ++i)
            #pragma unroll
            for (int j = i + 1; j < DIM; ++j) {
                const R o = g[i][j] + g[j][i];  // 2 e_ij
                off = fma(o, o, off);
            }
        st = fma(tr, tr, st);
        se += fma(R(0.5), off, dg);
        self_sums<R, T, DIM, TT + 1>(P, ih, Eb, st, se);
    }
}

// Sums over the voxel's elements of tr e tr f and e : f for the corner values
// Pe, Pf of two load cases, in arithmetic R.
template <typename R, typename T, int DIM, int TT = 0>
__device__ __forceinline__ void pair_sums(const T (&Pe)[1 << DIM][DIM], const T (&Pf)[1 << DIM][DIM], const T (&ih)[3],
                                          const R (&Ebe)[DIM][DIM], const R (&Ebf)[DIM][DIM], R &st, R &se) {
    constexpr int NEL = DIM == 3 ? 6 : 2;
    if constexpr (TT < NEL) {
        R ge[DIM][DIM], gf[DIM][DIM];
        element_grad<R, T, DIM, TT>(Pe, ih, Ebe, ge);
        element_grad<R, T, DIM, TT>(Pf, ih, Ebf, gf);
        R te = ge[0][0], tf = gf[0][0], dg = ge[0][0] * gf[0][0], off = R(0);
        #pragma unroll
        for (int i = 1; i < DIM; ++i) {
            te += ge[i][i];
            tf += gf[i][i];
            dg = fma(ge[i][i], gf[i][i], dg);
        }
        #pragma unroll
        for (int i = 0; i < DIM; ++i)
            #pragma unroll
            for (int j = i + 1; j < DIM; ++j) off = fma(ge[i][j] + ge[j][i], gf[i][j] + gf[j][i], off);
        st = fma(te, tf, st);
        se += fma(R(0.5), off, dg);
        pair_sums<R, T, DIM, TT + 1>(Pe, Pf, ih, Ebe, Ebf, st, se);
    }
}

// Stresses s = C e of the voxel's elements for corner values P: their sum
// over the elements into ss (symmetric storage as stress_of), the sum of
// e : s into w, the nodal forces F = B^T s of the voxel (so that
// sum_elements f : s = sum_c P'[c] . F[c] + Ebar' : ss for the strains f of
// any other corner values P' and mean strain Ebar'), and, when FIELDS, the
// full strain and stress blocks of element TT at fe + TT D^2, fs + TT D^2.
template <typename T, int DIM, bool FIELDS, int TT = 0>
__device__ __forceinline__ void element_forces(const T (&P)[1 << DIM][DIM], const T (&ih)[3],
                                               const double (&Eb)[DIM][DIM], double lam, double mu,
                                               double (&F)[1 << DIM][DIM], double (&ss)[DIM == 3 ? 6 : 3], double &w,
                                               T *fe, T *fs) {
    constexpr int NEL = DIM == 3 ? 6 : 2;
    constexpr int NS = DIM == 3 ? 6 : 3;
    if constexpr (TT < NEL) {
        double g[DIM][DIM];
        element_grad<double, T, DIM, TT>(P, ih, Eb, g);
        double sr[NS];
        const double m2 = 2.0 * mu;
        if constexpr (DIM == 3) {
            const double lt = lam * (g[0][0] + g[1][1] + g[2][2]);
            const double o0 = g[1][2] + g[2][1], o1 = g[0][2] + g[2][0], o2 = g[0][1] + g[1][0];  // 2 e_ij
            sr[0] = fma(m2, g[0][0], lt);
            sr[1] = fma(m2, g[1][1], lt);
            sr[2] = fma(m2, g[2][2], lt);
            sr[3] = mu * o0;
            sr[4] = mu * o1;
            sr[5] = mu * o2;
            w = fma(g[0][0], sr[0], w);
            w = fma(g[1][1], sr[1], w);
            w = fma(g[2][2], sr[2], w);
            w = fma(o0, sr[3], w);
            w = fma(o1, sr[4], w);
            w = fma(o2, sr[5], w);
            if constexpr (FIELDS) {
                const double e[6] = {g[0][0], g[1][1], g[2][2], 0.5 * o0, 0.5 * o1, 0.5 * o2};
                if (fe) put_full<T, DIM>(fe + TT * 9, e);
                if (fs) put_full<T, DIM>(fs + TT * 9, sr);
            }
        } else {
            const double lt = lam * (g[0][0] + g[1][1]);
            const double o2 = g[0][1] + g[1][0];
            sr[0] = fma(m2, g[0][0], lt);
            sr[1] = fma(m2, g[1][1], lt);
            sr[2] = mu * o2;
            w = fma(g[0][0], sr[0], w);
            w = fma(g[1][1], sr[1], w);
            w = fma(o2, sr[2], w);
            if constexpr (FIELDS) {
                const double e[3] = {g[0][0], g[1][1], 0.5 * o2};
                if (fe) put_full<T, DIM>(fe + TT * 4, e);
                if (fs) put_full<T, DIM>(fs + TT * 4, sr);
            }
        }
        #pragma unroll
        for (int k = 0; k < NS; ++k) ss[k] += sr[k];
        // F: the element's edge along axis a (corners c0 -> c1) carries the
        // gradient (P[c1] - P[c0]) / h_a, so s_ia / h_a goes to c1 and back from c0
        constexpr int BASE3[6][3] = {{0, 1, 3}, {0, 5, 1}, {2, 0, 3}, {6, 0, 2}, {4, 5, 0}, {6, 4, 0}};
        constexpr int BASE2[2][2] = {{0, 0}, {2, 1}};
        constexpr int SYM3[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
        constexpr int SYM2[2][2] = {{0, 2}, {2, 1}};
        #pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            const int c0 = DIM == 3 ? BASE3[TT][ax] : BASE2[TT][ax];
            const int c1 = c0 | (1 << ax);
            #pragma unroll
            for (int i = 0; i < DIM; ++i) {
                const double f = sr[DIM == 3 ? SYM3[i][ax] : SYM2[i][ax]] * double(ih[ax]);
                F[c1][i] += f;
                F[c0][i] -= f;
            }
        }
        element_forces<T, DIM, FIELDS, TT + 1>(P, ih, Eb, lam, mu, F, ss, w, fe, fs);
    }
}

// Workgroup (load case li of microstructure b, voxel tile, chunk):
// <sigma_l> partials, W_lm partials for m >= l, and the strain and stress
// fields of load case l when requested.  The stresses of the voxel's elements
// under load case l stay in registers while the later load cases' strains
// are formed against them.
template <typename T, int DIM, bool FIELDS>
__global__ __launch_bounds__(kThreads) void k_post_march(PK<T> a, MarchGeom geo) {
    using TL = MTile<DIM>;
    constexpr int NEL = DIM == 3 ? 6 : 2;
    constexpr int NS = DIM == 3 ? 6 : 3;
    __shared__ double red[kThreads / 64];
    const int G = a.G;
    int t = xcd_remap(blockIdx.x, (int)gridDim.x);
    const int li = t % G;
    t /= G;
    const int tz_t = t % geo.ntz;
    t /= geo.ntz;
    const int ty_t = t % geo.nty;
    const int ch = t / geo.nty;
    const int b = blockIdx.y;
    const int l = b * G + li;
    const int nl = G - li;  // pairs (l, l + k), k < nl
    const int y = ty_t * TL::VY + (DIM == 3 ? (int)threadIdx.x / TL::VZ : 0);
    const int z = tz_t * TL::VZ + (int)threadIdx.x % TL::VZ;
    const bool inside = (DIM == 2 || y < a.n1) && z < a.n2;
    const int x0 = ch * kMarchChunk, x1 = min(x0 + kMarchChunk, a.n0);
    const uint32_t plane = (uint32_t)a.n1 * (uint32_t)a.n2;
    const long long mo = (long long)b * a.N;
    double Ebl[DIM][DIM];
    ebar_full<DIM>(a.Ebar, l, Ebl);
    double sig[NS], w[kMarchG];
    #pragma unroll
    for (int k = 0; k < NS; ++k) sig[k] = 0.0;
    #pragma unroll
    for (int k = 0; k < kMarchG; ++k) w[k] = 0.0;
    if (inside) {
        ColumnCorners<DIM> cc;
        cc.init(a.n1, a.n2, DIM == 3 ? y : 0, z);
        const uint32_t vin = cc.o[0];
        for (int X = x0; X < x1; ++X) {
            const uint32_t xa = (uint32_t)X * plane, xb = (uint32_t)(X + 1 == a.n0 ? 0 : X + 1) * plane;
            const uint32_t v = xa + vin;
            const double lam = double(a.lam[mo + v]), mu = double(a.mu[mo + v]);
            T P[1 << DIM][DIM];
            if (a.u)
                column_corners<T, DIM>(a, l, xa, xb, cc, P);
            else
                for_corners_zero<T, DIM>(P);
            double F[1 << DIM][DIM], ss[NS];
            #pragma unroll
            for (int c = 0; c < (1 << DIM); ++c)
                #pragma unroll
                for (int i = 0; i < DIM; ++i) F[c][i] = 0.0;
            #pragma unroll
            for (int k = 0; k < NS; ++k) ss[k] = 0.0;
            if constexpr (FIELDS) {
                const long long off = ((long long)l * a.N + v) * NEL * DIM * DIM;
                element_forces<T, DIM, true>(P, a.ih, Ebl, lam, mu, F, ss, w[0], a.strain ? a.strain + off : nullptr,
                                             a.stress ? a.stress + off : nullptr);
            } else {
                element_forces<T, DIM, false>(P, a.ih, Ebl, lam, mu, F, ss, w[0], nullptr, nullptr);
            }
            #pragma unroll
            for (int k = 0; k < NS; ++k) sig[k] += ss[k];
            // W_lm for the later load cases m = l + k of the microstructure:
            // sum_elements e_m : s = sum_c u_m[c] . F[c] + Ebar_m : ss (one
            // pair at a time: not unrolled, so that the corner loads of the
            // later load cases are not all hoisted into registers)
            #pragma unroll 1
            for (int k = 1; k < nl; ++k) {
                const double *Em = a.Ebar + (l + k) * DIM * DIM;
                double acc;
                if constexpr (DIM == 3)
                    acc = Em[0] * ss[0] + Em[4] * ss[1] + Em[8] * ss[2] + 2.0 * (Em[5] * ss[3] + Em[2] * ss[4] + Em[1] * ss[5]);
                else
                    acc = Em[0] * ss[0] + Em[3] * ss[1] + 2.0 * Em[1] * ss[2];
                if (a.u) {
                    column_corners<T, DIM>(a, l + k, xa, xb, cc, P);
                    #pragma unroll
                    for (int c = 0; c < (1 << DIM); ++c)
                        #pragma unroll
                        for (int i = 0; i < DIM; ++i) acc = fma(double(P[c][i]), F[c][i], acc);
                }
                #pragma unroll
                for (int j = 1; j < kMarchG; ++j) w[j] += j == k ? acc : 0.0;
            }
        }
    }
    const int blk = (ch * geo.nty + ty_t) * geo.ntz + tz_t;
    for (int k = 0; k < NS; ++k) {
        const double sm = block_sum<kThreads>(sig[k], red);
        if (threadIdx.x == 0) a.partial[((long long)l * NS + k) * a.nblk + blk] = sm;
    }
    // pair (l, l + k) of microstructure b: pairs ordered l outer, m >= l inner
    const int pbase = a.L * NS + b * (G * (G + 1) / 2) + li * G - li * (li - 1) / 2;
    #pragma unroll
    for (int k = 0; k < kMarchG; ++k) {
        if (k < nl) {
            const double sm = block_sum<kThreads>(w[k], red);
            if (threadIdx.x == 0) a.partial[(long long)(pbase + k) * a.nblk + blk] = sm;
        }
    }
}

// Corner values of load case l on one node plane (in-plane corners
// (cy, cz) = 00, 10, 01, 11 in 3D, cz = 0, 1 in 2D) at plane offset xo.
// The plane's base address is uniform (scalar registers) and the in-plane
// byte offsets per thread fixed, so no address is formed per plane.
template <typename T, int DIM>
__device__ __forceinline__ void plane_corners(const PK<T> &a, int l, uint32_t xo, const uint32_t (&ob)[4],
                                              T (&C)[DIM == 3 ? 4 : 2][DIM]) {
    // one raw buffer over the plane per component: a uniform base and the
    // 32-bit lane offsets, no 64-bit address arithmetic per load
    const long long plane_bytes = (long long)a.n1 * a.n2 * (long long)sizeof(T);
    #pragma unroll
    for (int i = 0; i < DIM; ++i) {
        #pragma unroll
        for (int k = 0; k < (DIM == 3 ? 4 : 2); ++k)
            C[k][i] = a.u ? buffer_ld<T>(raw_buffer(a.u + ((long long)l * DIM + i) * a.N + xo, plane_bytes), ob[k]) : T(0);
    }
}

// Voxel corners (c = cx + 2 cy (+ 4 cz)) from the planes X (A) and X + 1 (B).
template <typename T, int DIM>
__device__ __forceinline__ void join_planes(const T (&A)[DIM == 3 ? 4 : 2][DIM], const T (&B)[DIM == 3 ? 4 : 2][DIM],
                                            T (&P)[1 << DIM][DIM]) {
    #pragma unroll
    for (int c = 0; c < (1 << DIM); ++c)
        #pragma unroll
        for (int i = 0; i < DIM; ++i) P[c][i] = (c & 1) ? B[c >> 1][i] : A[c >> 1][i];
}

// Workgroup (voxel tile, chunk, microstructure b): the sensitivity pairs of
// b (see k_sens).  Pairs outer, the chunk's planes inner: a load case's node
// plane X + 1 is carried in registers to the next voxel plane, so each node
// plane of a pair's load cases is read once per workgroup, and the working
// set of a workgroup is one or two load cases' planes (L2-resident for the
// neighbouring tiles that share its edge nodes).  The chunk's per-voxel sums
// stay in registers (the plane loop is unrolled).  OFFDIAG: the pair list
// holds pairs l != m (else every pair is diagonal, and the kernel keeps the
// registers of one load case only).
template <typename T, int DIM, bool OFFDIAG>
__global__ __launch_bounds__(kThreads) void k_sens_march(PK<T> a, MarchGeom geo, const int *pl, const int *pm,
                                                         const double *pw, const int *gofs, double scale, T *g_lam,
                                                         T *g_mu, T *g_E, double aE, double bE) {
    using TL = MTile<DIM>;
    constexpr int NK = DIM == 3 ? 4 : 2;
    int t = xcd_remap(blockIdx.x, (int)gridDim.x);
    const int tz_t = t % geo.ntz;
    t /= geo.ntz;
    const int ty_t = t % geo.nty;
    const int ch = t / geo.nty;
    const int b = blockIdx.y;
    const int y = ty_t * TL::VY + (DIM == 3 ? (int)threadIdx.x / TL::VZ : 0);
    const int z = tz_t * TL::VZ + (int)threadIdx.x % TL::VZ;
    if (!((DIM == 2 || y < a.n1) && z < a.n2)) return;
    const int x0 = ch * kMarchChunk, nx = min(kMarchChunk, a.n0 - x0);
    const uint32_t plane = (uint32_t)a.n1 * (uint32_t)a.n2;
    const int q0 = gofs[b], q1 = gofs[b + 1];
    ColumnCorners<DIM> cc;
    cc.init(a.n1, a.n2, DIM == 3 ? y : 0, z);
    uint32_t ob[4];  // in-plane byte offsets (n1 n2 sizeof(T) < 2^31: checked by the launcher)
    #pragma unroll
    for (int k = 0; k < 4; ++k) ob[k] = cc.o[k] * (uint32_t)sizeof(T);
    double gl[kMarchChunk], gm[kMarchChunk];
    #pragma unroll
    for (int k = 0; k < kMarchChunk; ++k) gl[k] = gm[k] = 0.0;
    // the voxel's element sums in the plan precision T, the pairs in FP64
    for (int q = q0; q < q1; ++q) {
        const int l = pl[q], m = pm[q];
        const double wq = pw[q];
        T Ebl[DIM][DIM];
        ebar_full<DIM>(a.Ebar, l, Ebl);
        T Al[NK][DIM];
        plane_corners<T, DIM>(a, l, (uint32_t)x0 * plane, ob, Al);
        if (!OFFDIAG || m == l) {
            // (tr e)^2 and e : e over the elements
            #pragma unroll
            for (int k = 0; k < kMarchChunk; ++k) {
                if (k < nx) {
                    const int X1 = x0 + k + 1 == a.n0 ? 0 : x0 + k + 1;
                    T Bl[NK][DIM], P[1 << DIM][DIM];
                    plane_corners<T, DIM>(a, l, (uint32_t)X1 * plane, ob, Bl);
                    join_planes<T, DIM>(Al, Bl, P);
                    T sl = T(0), se = T(0);
                    self_sums<T, T, DIM>(P, a.ih, Ebl, sl, se);
                    gl[k] += wq * double(sl);
                    gm[k] += 2.0 * wq * double(se);
                    #pragma unroll
                    for (int c = 0; c < NK; ++c)
                        #pragma unroll
                        for (int i = 0; i < DIM; ++i) Al[c][i] = Bl[c][i];
                }
                __builtin_amdgcn_sched_barrier(0);  // keep later planes' loads out of this step (registers)
            }
        } else if constexpr (OFFDIAG) {
            // tr e tr f and e : f over the elements of both load cases
            T Ebm[DIM][DIM];
            ebar_full<DIM>(a.Ebar, m, Ebm);
            T Am[NK][DIM];
            plane_corners<T, DIM>(a, m, (uint32_t)x0 * plane, ob, Am);
            #pragma unroll
            for (int k = 0; k < kMarchChunk; ++k) {
                if (k < nx) {
                    const int X1 = x0 + k + 1 == a.n0 ? 0 : x0 + k + 1;
                    T Bl[NK][DIM], Bm[NK][DIM], Pl[1 << DIM][DIM], Pm[1 << DIM][DIM];
                    plane_corners<T, DIM>(a, l, (uint32_t)X1 * plane, ob, Bl);
                    plane_corners<T, DIM>(a, m, (uint32_t)X1 * plane, ob, Bm);
                    join_planes<T, DIM>(Al, Bl, Pl);
                    join_planes<T, DIM>(Am, Bm, Pm);
                    T sl = T(0), se = T(0);
                    pair_sums<T, T, DIM>(Pl, Pm, a.ih, Ebl, Ebm, sl, se);
                    gl[k] += wq * double(sl);
                    gm[k] += 2.0 * wq * double(se);
                    #pragma unroll
                    for (int c = 0; c < NK; ++c)
                        #pragma unroll
                        for (int i = 0; i < DIM; ++i) {
                            Al[c][i] = Bl[c][i];
                            Am[c][i] = Bm[c][i];
                        }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    #pragma unroll
    for (int k = 0; k < kMarchChunk; ++k) {
        if (k < nx) {
            const long long v = (long long)b * a.N + (uint32_t)(x0 + k) * plane + cc.o[0];
            if (g_E) {
                g_E[v] = T((aE * gl[k] + bE * gm[k]) * scale);
            } else {
                g_lam[v] = T(gl[k] * scale);
                g_mu[v] = T(gm[k] * scale);
            }
        }
    }
}

__global__ void k_reduce_slots(const double *part, int nblk, double *out, double scale) {
    __shared__ double red[kThreads / 64];
    const int slot = blockIdx.x;
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kThreads) v += part[(long long)slot * nblk + i];
    const double s = block_sum<kThreads>(v, red);
    if (threadIdx.x == 0) out[slot] = s * scale;
}

template <typename T>
PK<T> post_args(const feh_plan &p) {
    PK<T> a{};
    a.lam = p.ptr<const T>(p.off_lam);
    a.mu = p.ptr<const T>(p.off_mu);
    if (p.dim == 3) {
        a.n0 = (int)p.n[0];
        a.n1 = (int)p.n[1];
        a.n2 = (int)p.n[2];
    } else {
        a.n0 = (int)p.n[0];
        a.n1 = 1;
        a.n2 = (int)p.n[1];
    }
    a.N = p.N;
    a.L = p.L;
    a.G = p.G;
    a.nbatch = p.nbatch;
    for (int i = 0; i < 3; ++i) a.ih[i] = T(1.0 / p.h[i]);
    a.nsym = p.dim == 3 ? 6 : 3;
    return a;
}

}  // namespace

// Does the plan take the plane-marching post-processing?
static bool march_ok(const feh_plan &p) {
    const double plane_bytes = (p.dim == 3 ? (double)p.n[1] * (double)p.n[2] : (double)p.n[1]) *
                               (p.prec == FEH_FP64 ? 8.0 : 4.0);
    return p.G <= kMarchG && plane_bytes < 2147483648.0;  // raw buffers over one plane
}

int post_num_parts(const feh_plan &p) {
    long long b = (p.N + kThreads - 1) / kThreads;
    if (b > 512) b = 512;
    if (march_ok(p)) {
        const MarchGeom g = p.dim == 3 ? march_geom<3>(p) : march_geom<2>(p);
        b = std::max(b, (long long)g.nty * g.ntz * g.nchunk);
    }
    return (int)b;
}

int post_num_slots(const feh_plan &p) {
    const int ns = p.dim == 3 ? 6 : 3;
    return p.L * ns + p.nbatch * (p.G * (p.G + 1) / 2);
}

template <typename T>
static int post_t(const feh_plan &p, const void *u, const double *Ebar, void *strain, void *stress, double *partial,
                  double *sums) {
    PK<T> a = post_args<T>(p);
    a.u = static_cast<const T *>(u);
    a.Ebar = Ebar;
    a.strain = static_cast<T *>(strain);
    a.stress = static_cast<T *>(stress);
    a.partial = partial;
    if (march_ok(p)) {
        const MarchGeom geo = p.dim == 3 ? march_geom<3>(p) : march_geom<2>(p);
        a.nblk = geo.nty * geo.ntz * geo.nchunk;
        dim3 g(a.nblk * p.G, p.nbatch);
        const bool fields = a.strain || a.stress;
        if (p.dim == 3 && fields)
            hipLaunchKernelGGL((k_post_march<T, 3, true>), g, dim3(kThreads), 0, p.stream, a, geo);
        else if (p.dim == 3)
            hipLaunchKernelGGL((k_post_march<T, 3, false>), g, dim3(kThreads), 0, p.stream, a, geo);
        else if (fields)
            hipLaunchKernelGGL((k_post_march<T, 2, true>), g, dim3(kThreads), 0, p.stream, a, geo);
        else
            hipLaunchKernelGGL((k_post_march<T, 2, false>), g, dim3(kThreads), 0, p.stream, a, geo);
    } else {
        const long long nb = (p.N + kThreads - 1) / kThreads;
        a.nblk = (int)(nb > 512 ? 512 : nb);
        const int nq = p.L + p.nbatch * (p.G * (p.G + 1) / 2);
        dim3 g(a.nblk, nq);
        if (p.dim == 3)
            hipLaunchKernelGGL((k_post<T, 3>), g, dim3(kThreads), 0, p.stream, a);
        else
            hipLaunchKernelGGL((k_post<T, 2>), g, dim3(kThreads), 0, p.stream, a);
    }
    int rc = hip_check(hipGetLastError(), "post launch");
    if (rc) return rc;
    const int ne = p.dim == 3 ? 6 : 2;
    hipLaunchKernelGGL(k_reduce_slots, dim3(post_num_slots(p)), dim3(kThreads), 0, p.stream, partial, a.nblk, sums,
                       1.0 / ((double)p.N * ne));
    return hip_check(hipGetLastError(), "post reduce");
}

int launch_post_sums(const feh_plan &p, const void *u, const double *Ebar_dev, void *strain, void *stress,
                     double *partial, double *sums) {
    return p.prec == FEH_FP64 ? post_t<double>(p, u, Ebar_dev, strain, stress, partial, sums)
                              : post_t<float>(p, u, Ebar_dev, strain, stress, partial, sums);
}

template <typename T>
static int grad_t(const feh_plan &p, const void *u, void *e) {
    PK<T> a = post_args<T>(p);
    a.u = static_cast<const T *>(u);
    a.strain = static_cast<T *>(e);
    a.grad_only = 1;
    long long g = (p.N + kThreads - 1) / kThreads;
    if (g > 65535) g = 65535;
    dim3 grid((unsigned)g, p.L);
    if (p.dim == 3)
        hipLaunchKernelGGL((k_grad<T, 3>), grid, dim3(kThreads), 0, p.stream, a);
    else
        hipLaunchKernelGGL((k_grad<T, 2>), grid, dim3(kThreads), 0, p.stream, a);
    return hip_check(hipGetLastError(), "grad launch");
}

int launch_grad(const feh_plan &p, const void *u, void *e) {
    return p.prec == FEH_FP64 ? grad_t<double>(p, u, e) : grad_t<float>(p, u, e);
}

template <typename T>
static int sens_t(const feh_plan &p, const void *u, const double *Ebar, const int *pl, const int *pm, const double *pw,
                  const int *gofs, bool offdiag, void *g_lam, void *g_mu, void *g_E, double aE, double bE) {
    PK<T> a = post_args<T>(p);
    a.u = static_cast<const T *>(u);
    a.Ebar = Ebar;
    long long g = (p.N + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    const int ne = p.dim == 3 ? 6 : 2;
    const double scale = 1.0 / ((double)p.N * ne);
    if (march_ok(p)) {
        const MarchGeom geo = p.dim == 3 ? march_geom<3>(p) : march_geom<2>(p);
        dim3 grid(geo.nty * geo.ntz * geo.nchunk, p.nbatch);
#define FEH_SENS(DV, OD)                                                                                     \
        hipLaunchKernelGGL((k_sens_march<T, DV, OD>), grid, dim3(kThreads), 0, p.stream, a, geo, pl, pm, pw, gofs, \
                           scale, static_cast<T *>(g_lam), static_cast<T *>(g_mu), static_cast<T *>(g_E), aE, bE)
        if (p.dim == 3) {
            if (offdiag) FEH_SENS(3, true);
            else FEH_SENS(3, false);
        } else {
            if (offdiag) FEH_SENS(2, true);
            else FEH_SENS(2, false);
        }
#undef FEH_SENS
        return hip_check(hipGetLastError(), "sensitivity launch");
    }
    if (p.dim == 3)
        hipLaunchKernelGGL((k_sens<T, 3>), dim3((unsigned)g), dim3(kThreads), 0, p.stream, a, pl, pm, pw, gofs, scale,
                           static_cast<T *>(g_lam), static_cast<T *>(g_mu), static_cast<T *>(g_E), aE, bE);
    else
        hipLaunchKernelGGL((k_sens<T, 2>), dim3((unsigned)g), dim3(kThreads), 0, p.stream, a, pl, pm, pw, gofs, scale,
                           static_cast<T *>(g_lam), static_cast<T *>(g_mu), static_cast<T *>(g_E), aE, bE);
    return hip_check(hipGetLastError(), "sensitivity launch");
}

int launch_sensitivity(const feh_plan &p, const void *u, const double *Ebar_dev, const int *pl, const int *pm,
                       const double *pw, const int *gofs, bool offdiag, void *g_lam, void *g_mu, void *g_E, double aE,
                       double bE) {
    return p.prec == FEH_FP64 ? sens_t<double>(p, u, Ebar_dev, pl, pm, pw, gofs, offdiag, g_lam, g_mu, g_E, aE, bE)
                              : sens_t<float>(p, u, Ebar_dev, pl, pm, pw, gofs, offdiag, g_lam, g_mu, g_E, aE, bE);
}

}  // namespace feh
