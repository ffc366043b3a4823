// Finite-element stencils on the structured grid: q = B^T C B p and friends.
//
// Discretisation (Sec. "Linear finite elements", small-strain appendix): each
// voxel holds n_e linear simplices (2 triangles in 2D, 6 Kuhn tetrahedra in
// 3D) with a constant strain e = sym(grad u) per element, stress
// sigma = lambda tr(e) I + 2 mu e and nodal force |e| B_e^T sigma.
//
// Both B and B^T are written in edge-difference form.  Every element
// gradient is built from differences of nodal values along voxel edges
// (G[:, a] = (u(end) - u(start)) / h_a), so constants map to exactly zero.
// Transposed, every element pushes the column sigma[:, a] |e| / h_a onto the
// voxel edge it used along axis a ("edge flux").  An edge of type (a, c)
// (axis a, start corner c inside its voxel) starting at node n belongs to
// voxel n - c, and the same edge type ending at n to voxel n - e_a - c, so
//   q(n) = sum_{a, c: c_a = 0} [ E_{a,c}(n - e_a - c) - E_{a,c}(n - c) ].
// Each bracket is a difference of the same quantity taken from two voxels:
// in a uniform region every bracket is exactly zero, so a uniform strain in
// a uniform material produces exactly zero force in any precision.
//
// Kernel layout: one workgroup evaluates a VY x VZ tile of voxels in the
// (axis 1, axis 2) plane, one voxel per thread, and marches along axis 0 over
// a chunk of planes.  The nodes it updates are those whose in-plane voxels
// all lie in the tile ((VY - 1) x (VZ - 1) in 3D, VZ - 1 in 2D); neighbouring
// tiles overlap by one voxel row and column, which keeps every wave on the
// same instruction stream (no extra round for halo voxels).  Per step the
// workgroup stages one node plane of the tile (one extra row and column of
// nodes) in LDS, each thread evaluates its voxel (edge fluxes into LDS), and
// each updated node combines the fluxes of its in-plane voxels; the terms
// whose voxels lie in the previous plane are carried in registers (two
// planes per loop trip, so that they alternate between two register sets).
// Global loads and stores go through raw buffers over one plane of one
// component; the lanes that update no node store past the buffer's end,
// which the hardware drops, so the node phase has no branch.  The fused CG
// variant accumulates p.q in FP64 for the step length (the update of p and u
// is fused into the last inverse FFT pass).
#include "device_common.hpp"

namespace feh {
namespace {

// Edge numbering: axis a, start corner c with c_a = 0; k enumerates the
// bits of the two other axes in increasing order (low bit first).
template <int A, int C>
struct EdgeK {
    static constexpr int b = A == 0 ? 1 : 0;
    static constexpr int d = A == 2 ? 1 : 2;
    static constexpr int k = ((C >> b) & 1) | (((C >> d) & 1) << 1);
};

// Strain (+ Ebar) -> stress -> edge fluxes of one tetrahedron with axis path
// (A0, A1, A2), from G[i][a] = d u_i / d x_a.  Eb = (xx, yy, zz, yz, xz, xy).
// E[(a * 4 + k) * 3 + i].  UNIT: all voxel sizes are 1 (no 1/h factors);
// EB: the macroscopic strain enters (right-hand side / residual only).
template <typename T, int A0, int A1, int A2, bool UNIT, bool EB>
__device__ __forceinline__ void tet_edges(const T (&G)[3][3], T lam, T mu, const T (&ih)[3], const T (&Eb)[6],
                                          T (&E)[36]) {
    constexpr int V1 = 1 << A0, V2 = V1 | (1 << A1);
    constexpr int k0 = EdgeK<A0, 0>::k, k1 = EdgeK<A1, V1>::k, k2 = EdgeK<A2, V2>::k;
    T e0 = G[0][0], e1 = G[1][1], e2 = G[2][2];
    if constexpr (EB) {
        e0 += Eb[0];
        e1 += Eb[1];
        e2 += Eb[2];
    }
    const T lt = lam * (e0 + e1 + e2), m2 = mu + mu;
    T S[3][3];
    S[0][0] = lt + m2 * e0;
    S[1][1] = lt + m2 * e1;
    S[2][2] = lt + m2 * e2;
    S[1][2] = S[2][1] = mu * (G[1][2] + G[2][1]);
    S[0][2] = S[2][0] = mu * (G[0][2] + G[2][0]);
    S[0][1] = S[1][0] = mu * (G[0][1] + G[1][0]);
    if constexpr (EB) {
        S[1][2] = S[2][1] = S[1][2] + m2 * Eb[3];
        S[0][2] = S[2][0] = S[0][2] + m2 * Eb[4];
        S[0][1] = S[1][0] = S[0][1] + m2 * Eb[5];
    }
    #pragma unroll
    for (int i = 0; i < 3; ++i) {
        if constexpr (UNIT) {
            E[(A0 * 4 + k0) * 3 + i] += S[i][A0];
            E[(A1 * 4 + k1) * 3 + i] += S[i][A1];
            E[(A2 * 4 + k2) * 3 + i] += S[i][A2];
        } else {
            E[(A0 * 4 + k0) * 3 + i] += S[i][A0] * ih[A0];
            E[(A1 * 4 + k1) * 3 + i] += S[i][A1] * ih[A1];
            E[(A2 * 4 + k2) * 3 + i] += S[i][A2] * ih[A2];
        }
    }
}

template <typename T, int A0, int A1, int A2, bool UNIT, bool EB>
__device__ __forceinline__ void tet_from_nodes(const T (&P)[8][3], T lam, T mu, const T (&ih)[3], const T (&Eb)[6],
                                               T (&E)[36]) {
    constexpr int V1 = 1 << A0, V2 = V1 | (1 << A1);
    T G[3][3];
    #pragma unroll
    for (int i = 0; i < 3; ++i) {
        G[i][A0] = P[V1][i] - P[0][i];
        G[i][A1] = P[V2][i] - P[V1][i];
        G[i][A2] = P[7][i] - P[V2][i];
        if constexpr (!UNIT) {
            G[i][A0] *= ih[A0];
            G[i][A1] *= ih[A1];
            G[i][A2] *= ih[A2];
        }
    }
    tet_edges<T, A0, A1, A2, UNIT, EB>(G, lam, mu, ih, Eb, E);
}

// All six tetrahedra of a voxel; lam, mu already carry the tetrahedron volume.
// The fluxes start at -0: x + (-0) = x exactly for every x (signed zeros
// included), so the first contribution to each edge folds into a move-free
// assignment, which +0 does not allow without relaxed floating-point rules.
template <typename T, bool UNIT, bool EB>
__device__ __forceinline__ void voxel3(const T (&P)[8][3], T lam, T mu, const T (&ih)[3], const T (&Eb)[6],
                                       T (&E)[36]) {
    #pragma unroll
    for (int j = 0; j < 36; ++j) E[j] = T(-0.0);
    tet_from_nodes<T, 0, 1, 2, UNIT, EB>(P, lam, mu, ih, Eb, E);
    tet_from_nodes<T, 0, 2, 1, UNIT, EB>(P, lam, mu, ih, Eb, E);
    tet_from_nodes<T, 1, 0, 2, UNIT, EB>(P, lam, mu, ih, Eb, E);
    tet_from_nodes<T, 1, 2, 0, UNIT, EB>(P, lam, mu, ih, Eb, E);
    tet_from_nodes<T, 2, 0, 1, UNIT, EB>(P, lam, mu, ih, Eb, E);
    tet_from_nodes<T, 2, 1, 0, UNIT, EB>(P, lam, mu, ih, Eb, E);
}

// Element field given directly (projection test export): fluxes of |e| sym(e_T).
template <typename T, int A0, int A1, int A2>
__device__ __forceinline__ void tet_div(const T *e, T vol, const T (&ih)[3], T (&E)[36]) {
    constexpr int V1 = 1 << A0, V2 = V1 | (1 << A1);
    constexpr int k0 = EdgeK<A0, 0>::k, k1 = EdgeK<A1, V1>::k, k2 = EdgeK<A2, V2>::k;
    #pragma unroll
    for (int i = 0; i < 3; ++i) {
        E[(A0 * 4 + k0) * 3 + i] += T(0.5) * vol * (e[i * 3 + A0] + e[A0 * 3 + i]) * ih[A0];
        E[(A1 * 4 + k1) * 3 + i] += T(0.5) * vol * (e[i * 3 + A1] + e[A1 * 3 + i]) * ih[A1];
        E[(A2 * 4 + k2) * 3 + i] += T(0.5) * vol * (e[i * 3 + A2] + e[A2 * 3 + i]) * ih[A2];
    }
}

// 2D: element 0 nodes 00,10,01 uses edges (x, c=0) and (y, c=0); element 1
// nodes 11,01,10 uses edges (x, c=e_y) and (y, c=e_x).  Corner index
// c = cx | c1 << 1.  E[(a * 2 + k) * 2 + i], k = offset along the other axis.
template <typename T>
__device__ __forceinline__ void tri_edges(T g00, T g01, T g10, T g11, T lam, T mu, T ihx, T ihy, const T (&Eb)[3],
                                          int kx, int ky, T (&E)[8]) {
    // g_ia = d u_i / d x_a
    const T e0 = g00 + Eb[0], e1 = g11 + Eb[1];
    const T lt = lam * (e0 + e1), m2 = mu + mu;
    const T sxy = mu * (g01 + g10) + m2 * Eb[2];
    E[(0 * 2 + kx) * 2 + 0] = (lt + m2 * e0) * ihx;
    E[(0 * 2 + kx) * 2 + 1] = sxy * ihx;
    E[(1 * 2 + ky) * 2 + 0] = sxy * ihy;
    E[(1 * 2 + ky) * 2 + 1] = (lt + m2 * e1) * ihy;
}

template <typename T>
__device__ __forceinline__ void voxel2(const T (&P)[4][2], T lam, T mu, T ihx, T ihy, const T (&Eb)[3], T (&E)[8]) {
    // element 0: d/dx = (P10 - P00) ihx, d/dy = (P01 - P00) ihy
    tri_edges<T>((P[1][0] - P[0][0]) * ihx, (P[2][0] - P[0][0]) * ihy, (P[1][1] - P[0][1]) * ihx,
                 (P[2][1] - P[0][1]) * ihy, lam, mu, ihx, ihy, Eb, 0, 0, E);
    // element 1: d/dx = (P11 - P01) ihx, d/dy = (P11 - P10) ihy
    tri_edges<T>((P[3][0] - P[2][0]) * ihx, (P[3][0] - P[1][0]) * ihy, (P[3][1] - P[2][1]) * ihx,
                 (P[3][1] - P[1][1]) * ihy, lam, mu, ihx, ihy, Eb, 1, 1, E);
}

template <typename T>
__device__ __forceinline__ void voxel2_div(const T *e, T vol, T ihx, T ihy, T (&E)[8]) {
    // e: [2 elements][2][2]
    #pragma unroll
    for (int el = 0; el < 2; ++el) {
        const T *ee = e + el * 4;
        const T sxy = T(0.5) * vol * (ee[1] + ee[2]);
        E[(0 * 2 + el) * 2 + 0] = vol * ee[0] * ihx;
        E[(0 * 2 + el) * 2 + 1] = sxy * ihx;
        E[(1 * 2 + el) * 2 + 0] = sxy * ihy;
        E[(1 * 2 + el) * 2 + 1] = vol * ee[3] * ihy;
    }
}

template <typename T>
struct SK {
    const T *in0;      // p / u
    T *out0;           // q / r
    const T *lam;
    const T *mu;
    const double *Ebar;
    double *partial;
    const LcState *st;
    int n0, n1, n2;    // 2D: n1 = 1, n2 = n[1]
    long long N;
    int xc, nchunk, nty, ntz, total;
    int part_stride;
    T ih[3];
    T vol;
    int ident;         // lambda = 0, mu = 1/2 everywhere
    int G;             // load cases per microstructure (material of load case l: l / G)
};

// Tile shapes: VY x VZ voxels per workgroup (one per thread).  HY = 1 when
// the tile has an axis-1 extent (3D); the node plane of the tile is
// (VY + HY) x (VZ + 1), the updated nodes advance by SY x SZ between tiles.
// 3D tiles are 8 or 16 rows of 32 voxels (256 or 512 threads): the taller
// tile re-reads fewer halo nodes ((VY + 1) 33 loaded per (VY - 1) 31 updated)
// at twice the LDS of the edge-flux exchange.
template <int DIM, int VYT>
struct Tile;
template <int VYT>
struct Tile<3, VYT> {
    static constexpr int VY = VYT, VZ = 32, HY = 1, NC = 3, NEDGE = 12;
    static constexpr int SY = VY - 1, SZ = VZ - 1, NT = VY * VZ;
};
template <int VYT>
struct Tile<2, VYT> {
    static constexpr int VY = 1, VZ = 256, HY = 0, NC = 2, NEDGE = 4;
    static constexpr int SY = 1, SZ = VZ - 1, NT = 256;
};

// The value held by lane - 1 of the wavefront (DPP shift of the whole wave
// right by one lane; lane 0, which has no source lane, receives zero through
// the bound control, so no register has to be zeroed for it).  In the 3D tile
// a row of 32 voxels lies inside one wavefront, so lane - 1 holds the voxel
// at z - 1.
__device__ __forceinline__ int lane_shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float from_left(float v) {
    return __builtin_bit_cast(float, lane_shr1(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_left(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)lane_shr1((int)(unsigned)b), hi = (unsigned)lane_shr1((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T, int DIM, int MODE, bool UNIT, int VYT>
__global__ __launch_bounds__((Tile<DIM, VYT>::NT)) void k_stencil(SK<T> a) {
    using TL = Tile<DIM, VYT>;
    constexpr int VY = TL::VY, VZ = TL::VZ, HY = TL::HY, NC = TL::NC, NEDGE = TL::NEDGE;
    constexpr int EY = VY + HY, EZ = VZ + 1;     // node plane of the tile
    constexpr int NE = EY * EZ, NT = TL::NT;
    constexpr int NQ = NEDGE * NC;               // edge-flux values per voxel
    constexpr int NSE = (NE + NT - 1) / NT;      // node-plane slots per thread
    static_assert(VY * VZ == NT, "one voxel per thread");
    static_assert(DIM == 2 || VZ == 32, "3D: one row of voxels per half wavefront");
    __shared__ T Pl[NC][NE];                     // one node plane
    // edge fluxes passed through LDS, one column per voxel: in 3D only the 24
    // values the next row of voxels needs (the left neighbour's come by DPP)
    constexpr int NX = DIM == 3 ? 24 : NQ;
    __shared__ T Es[NX][NT];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    int t = xcd_remap(blockIdx.x, a.total);
    const int tz_t = t % a.ntz;
    t /= a.ntz;
    const int ty_t = t % a.nty;
    t /= a.nty;
    const int ch = t % a.nchunk;
    const int lc = t / a.nchunk;
    const int blk_in_lc = (ch * a.nty + ty_t) * a.ntz + tz_t;

    // load cases that have stopped iterating
    if constexpr (MODE == ST_CG) {
        if (!a.st[lc].active) return;
    }
    T Eb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if constexpr (MODE == ST_RESID) {
        const double *E = a.Ebar + lc * DIM * DIM;
        if constexpr (DIM == 3) {
            Eb[0] = T(E[0]); Eb[1] = T(E[4]); Eb[2] = T(E[8]);
            Eb[3] = T(E[5]); Eb[4] = T(E[2]); Eb[5] = T(E[1]);
        } else {
            Eb[0] = T(E[0]); Eb[1] = T(E[3]); Eb[2] = T(E[1]);
        }
    }

    // in-plane origin of the tile's node plane (extended index (0, 0)); the
    // updated nodes start one row (3D) and one column further on
    const int y0 = ty_t * TL::SY - HY, z0 = tz_t * TL::SZ - 1;
    const int x0 = ch * a.xc;
    const int x1 = min(x0 + a.xc, a.n0);
    const long long N = a.N;
    const long long plane = (long long)a.n1 * a.n2;
    const long long lcoff = (long long)lc * NC * N;
    const long long moff = (long long)(lc / a.G) * N;  // this load case's microstructure
    const int ty = tid / VZ, tz = tid - (tid / VZ) * VZ;
    // the thread's voxel has its origin at node (ty, tz) of the tile; that
    // node is updated here when all of its in-plane voxels are in the tile
    const bool owner = ty >= HY && tz >= 1 && y0 + ty < a.n1 && z0 + tz < a.n2;

    // ---- per-thread node slots, fixed for the whole march.  Slot 0 is the
    // thread's own node; later slots cover the last row and column.
    int e_lds[NSE];        // extended node index (an unused slot repeats slot 0)
    unsigned e_boff[NSE];  // in-plane byte offset (the launcher checks that a plane fits 31 bits)
    #pragma unroll
    for (int s = 0; s < NSE; ++s) {
        int ey = -1, ez = -1;
        if (s == 0) {
            ey = ty;
            ez = tz;
        } else {
            const int hh = tid + (s - 1) * NT;  // extra node number
            constexpr int NH = NE - NT;
            if (hh < NH) {
                if constexpr (HY == 0) {
                    ey = 0;  // single row: its last node
                    ez = EZ - 1;
                } else if (hh < EZ) {
                    ey = EY - 1;  // last row
                    ez = hh;
                } else {
                    ey = hh - EZ;  // last column, rows 0 .. EY - 2
                    ez = EZ - 1;
                }
            }
        }
        if (ey >= 0) {
            e_lds[s] = ey * EZ + ez;
            e_boff[s] = (unsigned)(wrap(y0 + ey, a.n1) * a.n2 + wrap(z0 + ez, a.n2)) * (unsigned)sizeof(T);
        } else {
            // unused: its loads re-read the own node and its LDS store
            // repeats the own node's, same value to the same place
            e_lds[s] = e_lds[0];
            e_boff[s] = e_boff[0];
        }
    }
    const long long v_off = (long long)wrap(y0 + ty, a.n1) * a.n2 + wrap(z0 + tz, a.n2);
    const unsigned v_boff = (unsigned)v_off * (unsigned)sizeof(T);
    // node loads and stores go through raw buffers over one plane of one
    // component; a lane that updates no node stores past the buffer's end,
    // which the hardware drops, so no branch splits the node phase
    const unsigned st_boff = owner ? e_boff[0] : 0x80000000u;
    const long long plane_bytes = plane * (long long)sizeof(T);

    // ---- prefetch registers: node plane P and the material of one voxel
    // plane.  Every load is unconditional (unused slots and planes past the
    // chunk re-read valid addresses).
    T rz[NSE][NC];
    T mlam = T(0), mmu = T(0);
    auto fetch_nodes = [&](int P) __attribute__((always_inline)) {
        const long long base = lcoff + (long long)wrap(P, a.n0) * plane;
        #pragma unroll
        for (int s = 0; s < NSE; ++s) {
            #pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (MODE == ST_APPLY || MODE == ST_CG) {
                    rz[s][c] = buffer_ld<T>(raw_buffer(a.in0 + base + c * N, plane_bytes), e_boff[s]);
                } else if constexpr (MODE == ST_RESID) {
                    rz[s][c] = a.in0 ? buffer_ld<T>(raw_buffer(a.in0 + base + c * N, plane_bytes), e_boff[s]) : T(0);
                }
            }
        }
    };
    // stage the fetched node plane in LDS (one plane only: the previous plane's corners
    // stay in registers); returns the thread's own node value in own[]
    T own[NC];
    auto commit_nodes = [&]() __attribute__((always_inline)) {
        #pragma unroll
        for (int s = 0; s < NSE; ++s) {
            #pragma unroll
            for (int c = 0; c < NC; ++c) {
                Pl[c][e_lds[s]] = rz[s][c];
                if (s == 0) own[c] = rz[s][c];
            }
        }
    };
    auto fetch_material = [&](int V) __attribute__((always_inline)) {
        const long long base = moff + (long long)wrap(V, a.n0) * plane;
        mlam = buffer_ld<T>(raw_buffer(a.lam + base, plane_bytes), v_boff);  // unused (but allocated) for the identity material
        mmu = buffer_ld<T>(raw_buffer(a.mu + base, plane_bytes), v_boff);
    };

    // in-plane corners of the thread's voxel: k = cy + 2 cz (3D), k = cz (2D);
    // Pc holds them in the lower node plane of the current voxel plane
    constexpr int NK = DIM == 3 ? 4 : 2;
    T Pc[NK][NC];
    auto corner_lds = [&](int k) { return DIM == 3 ? (ty + (k & 1)) * EZ + tz + (k >> 1) : tz + k; };

    // carried terms: raw axis-0 edge fluxes of the previous voxel plane, and
    // the differences of the other axes' edges whose voxels lie in the
    // previous plane
    constexpr int NXE = DIM == 3 ? 4 : 2;  // axis-0 edges per voxel
    T cx[NXE * NC];
    T cq[NC];
    #pragma unroll
    for (int j = 0; j < NXE * NC; ++j) cx[j] = T(0);
    #pragma unroll
    for (int c = 0; c < NC; ++c) cq[c] = T(0);
    double acc = 0.0;

    if constexpr (MODE != ST_DIV) {
        fetch_nodes(x0 - 1);
        commit_nodes();
        fetch_nodes(x0);
        __syncthreads();
        #pragma unroll
        for (int k = 0; k < NK; ++k) {
            #pragma unroll
            for (int c = 0; c < NC; ++c) Pc[k][c] = (k == 0) ? own[c] : Pl[c][corner_lds(k)];
        }
        __syncthreads();
    }
    fetch_material(x0 - 1);

    // voxel column of the node's in-plane voxels at offset (-dy, -dz); threads
    // that update no node read an interior column instead (results unused)
    const int vo = (ty >= HY && tz >= 1) ? tid : HY * VZ + 1;
    auto vix = [&](int dy, int dz) { return vo - dy * VZ - dz; };

    // one step of the march: the voxels of plane X, then the nodes of plane X
    // (the first step, plane x0 - 1, only primes the carried terms)
    auto step = [&](const int X, auto first) __attribute__((always_inline)) {
        constexpr bool FIRST = decltype(first)::value;
        // ---- stage plane X+1, prefetch plane X+2 and the material of voxel plane X+1
        if constexpr (MODE != ST_DIV) commit_nodes();
        const T clam = mlam, cmu = mmu;
        if constexpr (MODE != ST_DIV) fetch_nodes(min(X + 2, x1));
        fetch_material(min(X + 1, x1 - 1));
        __syncthreads();
        // ---- voxel phase: the thread's voxel in plane X
        T pown[NC];  // p at the thread's own node of plane X
        T q[NC], nq[NC];
        #pragma unroll
        for (int i = 0; i < NC; ++i) {
            q[i] = cq[i];
            nq[i] = T(-0.0);  // x + (-0) = x: the first term folds into a move
        }
        T oy[12];    // 3D: the own voxel's axis-1 edge fluxes, kept for the node phase
        {
            T lam, mu;
            if (a.ident) {
                lam = T(0);
                mu = T(0.5) * a.vol;
            } else {
                lam = clam * a.vol;
                mu = cmu * a.vol;
            }
            if constexpr (DIM == 3) {
                T E[36];
                if constexpr (MODE == ST_DIV) {
                    const long long vidx = (long long)wrap(X, a.n0) * plane + v_off;
                    const T *e = a.in0 + ((long long)lc * N + vidx) * 54;
                    #pragma unroll
                    for (int j = 0; j < 36; ++j) E[j] = T(0);
                    tet_div<T, 0, 1, 2>(e + 0, a.vol, a.ih, E);
                    tet_div<T, 0, 2, 1>(e + 9, a.vol, a.ih, E);
                    tet_div<T, 1, 0, 2>(e + 18, a.vol, a.ih, E);
                    tet_div<T, 1, 2, 0>(e + 27, a.vol, a.ih, E);
                    tet_div<T, 2, 0, 1>(e + 36, a.vol, a.ih, E);
                    tet_div<T, 2, 1, 0>(e + 45, a.vol, a.ih, E);
                } else {
                    // corner c = cx + 2 cy + 4 cz; cx = 0 from registers, cx = 1 staged
                    T P[8][3];
                    #pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        #pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            P[2 * k][i] = Pc[k][i];
                            P[2 * k + 1][i] = (k == 0) ? own[i] : Pl[i][corner_lds(k)];
                        }
                    }
                    voxel3<T, UNIT, MODE == ST_RESID>(P, lam, mu, a.ih, Eb, E);
                    #pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        #pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            if (k == 0) pown[i] = Pc[0][i];
                            Pc[k][i] = P[2 * k + 1][i];
                        }
                    }
                }
                // export the fluxes the row below needs: x1, x3, y0..y3, z2, z3
                #pragma unroll
                for (int j = 0; j < 24; ++j) Es[j][tid] = E[j < 6 ? (j < 3 ? 3 + j : 6 + j) : (j < 18 ? 6 + j : 12 + j)];
                #pragma unroll
                for (int j = 0; j < 12; ++j) oy[j] = E[12 + j];
                // terms of the own voxel (x-edge c = 0) and of the left voxel
                // (x-edge c = (0,0,1), z-edges c = (x,0,0) paired with the own voxel),
                // the latter formed by lane - 1, which holds that voxel
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const T c0 = E[0 + i];
                    q[i] += cx[0 * 3 + i] - c0;
                    cx[0 * 3 + i] = c0;
                    const T c2 = E[6 + i];
                    const T d2 = cx[2 * 3 + i] - c2;
                    cx[2 * 3 + i] = c2;
                    q[i] += from_left(d2);
                    q[i] += from_left(E[24 + i]) - E[24 + i];
                    nq[i] += from_left(E[27 + i]) - E[27 + i];
                }
            } else {
                T E[8];
                if constexpr (MODE == ST_DIV) {
                    const long long vidx = (long long)wrap(X, a.n0) * plane + v_off;
                    voxel2_div<T>(a.in0 + ((long long)lc * N + vidx) * 8, a.vol, a.ih[0], a.ih[1], E);
                } else {
                    // corner c = cx + 2 cz
                    T P[4][2];
                    #pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        #pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            P[2 * k][i] = Pc[k][i];
                            P[2 * k + 1][i] = (k == 0) ? own[i] : Pl[i][corner_lds(k)];
                        }
                    }
                    const T Eb2[3] = {Eb[0], Eb[1], Eb[2]};
                    voxel2<T>(P, lam, mu, a.ih[0], a.ih[1], Eb2, E);
                    #pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        #pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            if (k == 0) pown[i] = Pc[0][i];
                            Pc[k][i] = P[2 * k + 1][i];
                        }
                    }
                }
                #pragma unroll
                for (int j = 0; j < 8; ++j) Es[j][tid] = E[j];
            }
        }
        __syncthreads();
        // ---- node phase (the thread's own node)
        {
            if constexpr (DIM == 3) {
                // fluxes of the voxel above (row ty - 1); row 0 reads its own
                // column (it updates no node and feeds no neighbour that does)
                const int ia = ty >= 1 ? tid - VZ : tid;
                T A[24];
                #pragma unroll
                for (int j = 0; j < 24; ++j) A[j] = Es[j][ia];
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    // x-edges c = (0,1,0) (voxel above) and c = (0,1,1) (above-left, from lane - 1)
                    const T c1 = A[0 + i];
                    q[i] += cx[1 * 3 + i] - c1;
                    cx[1 * 3 + i] = c1;
                    const T c3 = A[3 + i];
                    const T d3 = cx[3 * 3 + i] - c3;
                    cx[3 * 3 + i] = c3;
                    q[i] += from_left(d3);
                    // y-edges: above - own (k = 0, 1); above-left - left (k = 2, 3) from lane - 1
                    q[i] += A[6 + i] - oy[0 + i];
                    nq[i] += A[9 + i] - oy[3 + i];
                    q[i] += from_left(A[12 + i] - oy[6 + i]);
                    nq[i] += from_left(A[15 + i] - oy[9 + i]);
                    // z-edges: above-left (from lane - 1) - above (k = 2, 3)
                    q[i] += from_left(A[18 + i]) - A[18 + i];
                    nq[i] += from_left(A[21 + i]) - A[21 + i];
                }
            } else {
                // axis-0 edges: c = (0, c1), k = c1
                #pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int v = vix(0, k);
                    #pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const T cur = Es[(0 * 2 + k) * 2 + i][v];
                        q[i] += cx[k * 2 + i] - cur;
                        cx[k * 2 + i] = cur;
                    }
                }
                // axis-1 edges: c = (cx, 0), k = cx; voxels n - e_1 - c and n - c
                const int vlo = vix(0, 1), vhi = vix(0, 0);
                #pragma unroll
                for (int i = 0; i < 2; ++i) {
                    q[i] += Es[(1 * 2 + 0) * 2 + i][vlo] - Es[(1 * 2 + 0) * 2 + i][vhi];
                    nq[i] += Es[(1 * 2 + 1) * 2 + i][vlo] - Es[(1 * 2 + 1) * 2 + i][vhi];
                }
            }
            if constexpr (!FIRST) {
                #pragma unroll
                for (int i = 0; i < NC; ++i) {
                    buffer_st<T>(raw_buffer(a.out0 + lcoff + i * N + (long long)X * plane, plane_bytes), st_boff,
                                 MODE == ST_RESID ? -q[i] : q[i]);
                    // p.q of every lane (finite values); the lanes that own no
                    // node drop their sum at the end
                    if constexpr (MODE == ST_CG) acc += double(pown[i]) * double(q[i]);
                }
            }
            #pragma unroll
            for (int i = 0; i < NC; ++i) {
                // formed here, next to the lane shifts that feed it, rather
                // than sunk past the march's exit test into the next step
                asm volatile("" : "+v"(nq[i]));
                cq[i] = nq[i];
            }
        }
    };
    // two steps per trip, so that the values carried from one step to the
    // next alternate between two register sets instead of being copied
    step(x0 - 1, std::true_type{});
    for (int X = x0;; X += 2) {
        step(X, std::false_type{});
        if (X + 1 >= x1) break;
        step(X + 1, std::false_type{});
        if (X + 2 >= x1) break;
    }
    if constexpr (MODE == ST_CG) {
        if (!owner) acc = 0.0;
        const double s = block_sum<NT>(acc, red);
        if (tid == 0) a.partial[(long long)lc * a.part_stride + blk_in_lc] = s;
    }
}

// Planes per workgroup march: 32 in 3D; 8 in 2D, whose grids are small enough
// that the march length (not HBM) bounds a launch once most load cases of a
// batch have converged.
int xchunk(int n0, int dim) {
    const int c = dim == 3 ? 32 : 8;
    return n0 < c ? n0 : c;
}

template <typename T, int DIM, int VYT>
int launch_t(const feh_plan &p, int mode, const StencilArgs &sa) {
    using TL = Tile<DIM, VYT>;
    SK<T> a{};
    a.in0 = static_cast<const T *>(sa.in0);
    a.out0 = static_cast<T *>(sa.out0);
    a.lam = p.ptr<const T>(p.off_lam);
    a.mu = p.ptr<const T>(p.off_mu);
    a.Ebar = sa.Ebar;
    a.partial = sa.partial;
    a.st = sa.state;
    a.ident = sa.identity_material ? 1 : 0;
    a.G = p.G;
    if (DIM == 3) {
        a.n0 = (int)p.n[0];
        a.n1 = (int)p.n[1];
        a.n2 = (int)p.n[2];
        a.ih[0] = T(1.0 / p.h[0]);
        a.ih[1] = T(1.0 / p.h[1]);
        a.ih[2] = T(1.0 / p.h[2]);
        a.vol = T(sa.unit_volume ? 1.0 / 6.0 : p.h[0] * p.h[1] * p.h[2] / 6.0);
    } else {
        a.n0 = (int)p.n[0];
        a.n1 = 1;
        a.n2 = (int)p.n[1];
        a.ih[0] = T(1.0 / p.h[0]);
        a.ih[1] = T(1.0 / p.h[1]);
        a.ih[2] = T(1);
        a.vol = T(sa.unit_volume ? 0.5 : p.h[0] * p.h[1] / 2.0);
    }
    // in-plane byte offsets are 32-bit and the store buffers span one plane
    // (at most 4096^2 values: 128 MiB in FP64)
    if ((long long)a.n1 * a.n2 * (long long)sizeof(T) >= (1LL << 31))
        return set_error(FEH_EINVAL, "stencil: one plane of a field must stay below 2 GiB");
    a.N = p.N;
    a.xc = xchunk(a.n0, DIM);
    a.nchunk = (a.n0 + a.xc - 1) / a.xc;
    a.nty = (a.n1 + TL::SY - 1) / TL::SY;
    a.ntz = (a.n2 + TL::SZ - 1) / TL::SZ;
    a.total = p.L * a.nchunk * a.nty * a.ntz;
    a.part_stride = (int)p.part_stride;
    dim3 grid(a.total), block(TL::NT);
    const bool unit = p.h[0] == 1.0 && p.h[1] == 1.0 && (DIM == 2 || p.h[2] == 1.0);
#define FEH_STENCIL_CASE(M)                                                                                   \
    case M:                                                                                                   \
        if (unit) hipLaunchKernelGGL((k_stencil<T, DIM, M, true, VYT>), grid, block, 0, p.stream, a);             \
        else hipLaunchKernelGGL((k_stencil<T, DIM, M, false, VYT>), grid, block, 0, p.stream, a);                 \
        break;
    switch (mode) {
        FEH_STENCIL_CASE(ST_APPLY)
        FEH_STENCIL_CASE(ST_CG)
        FEH_STENCIL_CASE(ST_RESID)
        FEH_STENCIL_CASE(ST_DIV)
    default: return set_error(FEH_EINVAL, "bad stencil mode");
    }
#undef FEH_STENCIL_CASE
    return hip_check(hipGetLastError(), "stencil launch");
}

}  // namespace

int stencil_rows(const feh_plan &p) {
    if (p.dim != 3) return 1;
    if (p.tune_stencil_vy == 8 || p.tune_stencil_vy == 16) return p.tune_stencil_vy;
    return 8;
}

int stencil_num_parts(const feh_plan &p) {
    const int n0 = (int)p.n[0];
    const int xc = xchunk(n0, p.dim);
    const int nchunk = (n0 + xc - 1) / xc;
    if (p.dim == 3) {
        const int sy = stencil_rows(p) - 1, sz = 31;
        return nchunk * (int)((p.n[1] + sy - 1) / sy) * (int)((p.n[2] + sz - 1) / sz);
    }
    return nchunk * (int)((p.n[1] + Tile<2, 1>::SZ - 1) / Tile<2, 1>::SZ);
}

int launch_stencil(const feh_plan &p, int mode, const StencilArgs &a) {
    if (p.dim == 2)
        return p.prec == FEH_FP64 ? launch_t<double, 2, 1>(p, mode, a) : launch_t<float, 2, 1>(p, mode, a);
    if (stencil_rows(p) == 16)
        return p.prec == FEH_FP64 ? launch_t<double, 3, 16>(p, mode, a) : launch_t<float, 3, 16>(p, mode, a);
    return p.prec == FEH_FP64 ? launch_t<double, 3, 8>(p, mode, a) : launch_t<float, 3, 8>(p, mode, a);
}

}  // namespace feh
