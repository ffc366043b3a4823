// Batched Stockham FFTs staged through LDS, and the per-wavevector
// projection core (B^*B)^-1 fused into the first-axis pass.
//
// The transform pair follows the discrete Fourier transform appendix of the
// paper: forward sum_r f(r) exp(-i k.r) (unnormalised), inverse with 1/N.
// Real fields are transformed along the last (contiguous) axis to the half
// spectrum n_last/2 + 1 (two real samples packed into one complex point and
// untangled with a post-twiddle when n_last is even), then complex-to-complex
// along the other axes.  The spectrum of load case l is stored as
// [n0][(n1)][nh][D], components innermost, so the first-axis pass can read
// all D components of a wavevector in one coalesced segment.
//
// Stockham autosort (each pass reads the previous pass's output layout and
// writes the next, natural order at the end, no bit reversal): pass with
// radix R after earlier radices of product L*, L = L* R, m = n / L:
//   y[q + m (p + L* d)] = sum_c exp(-2 pi i c d / R) w_n^{c p m} x[q + c m + m R p]
// for q < m, p < L*, d < R.
#include <algorithm>

#include "device_common.hpp"

namespace feh {
namespace {

constexpr int kFftThreads = 256;

template <typename T>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) { return {a.y, -a.x}; }  // a * (-i)
template <typename T>
__device__ __forceinline__ Cx<T> mul_pi(Cx<T> a) { return {-a.y, a.x}; }  // a * (+i)
template <typename T>
__device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }

template <typename T>
__device__ __forceinline__ Cx<T> twid(const Cx<T> *tw, int tws, int e, bool inv) {
    Cx<T> w = tw[e * tws];
    if (inv) w.y = -w.y;
    return w;
}

// Dynamic LDS holds the twiddle table of the transformed axis (and, in the
// fused first-axis pass, the phase factors of the block's inner wavevector
// indices): staged once per workgroup so the butterflies never wait on global
// memory.
extern __shared__ double feh_dyn_lds[];

// FP64 transforms of general lengths (radix 3..13 and direct passes) are held
// to at most 256 VGPRs, two waves per SIMD; with tiles sized to the pass, two
// workgroups then fit a CU for rows of up to about 1700 points.
template <typename T, bool GEN>
constexpr int kGenWaves = (GEN && sizeof(T) == 8) ? 2 : 1;

// LDS one workgroup may hold on gfx950 (160 KiB).  Every launch checks its
// static plus dynamic LDS against it on the host and reports FEH_ENOTSUP
// instead of dispatching a workgroup the hardware cannot allocate.
constexpr size_t kLdsPerWorkgroup = 160 * 1024;

// Streaming global accesses with the nontemporal hint.  The last inverse pass
// uses them for p, u and z: it reads and writes each element of those fields
// once, and nothing reads them again before the next operator pass.  Measured
// per pass, the hint pays only there: on the forward pass (q fresh from the
// stencil) and on the spectrum passes it made the kernels slower.
template <typename T>
__device__ __forceinline__ Cx<T> ldc_nt(const Cx<T> *p) {
    typedef T V __attribute__((ext_vector_type(2)));
    const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    return Cx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void stc_nt(Cx<T> *p, Cx<T> c) {
    typedef T V __attribute__((ext_vector_type(2)));
    V v;
    v.x = c.x;
    v.y = c.y;
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}
template <typename T>
__device__ __forceinline__ T ldr_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void str_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }

template <typename T>
__device__ __forceinline__ void stage(T *dst, const T *src, int count) {
    for (int i = threadIdx.x; i < count; i += kFftThreads) dst[i] = src[i];
}

// In-place DFT of length R on registers: x[d] <- sum_c x[c] exp(-+2 pi i c d / R).
template <typename T, int R>
struct Dft {
    // generic radix (7, 11, 13): roots from the table of the full length n
    static __device__ __forceinline__ void run(Cx<T> (&x)[R], bool inv, const Cx<T> *tw, int tws, int n) {
        Cx<T> y[R];
        const int step = n / R;
        #pragma unroll
        for (int d = 0; d < R; ++d) {
            Cx<T> s = x[0];
            #pragma unroll
            for (int c = 1; c < R; ++c) s = cadd(s, cmul(x[c], twid(tw, tws, ((c * d) % R) * step, inv)));
            y[d] = s;
        }
        #pragma unroll
        for (int d = 0; d < R; ++d) x[d] = y[d];
    }
};

template <typename T>
struct Dft<T, 2> {
    static __device__ __forceinline__ void run(Cx<T> (&x)[2], bool, const Cx<T> *, int, int) {
        const Cx<T> a = x[0];
        x[0] = cadd(a, x[1]);
        x[1] = csub(a, x[1]);
    }
};

template <typename T>
struct Dft<T, 3> {
    static __device__ __forceinline__ void run(Cx<T> (&x)[3], bool inv, const Cx<T> *, int, int) {
        const T s3 = T(0.86602540378443864676);
        const Cx<T> t1 = cadd(x[1], x[2]), t2 = csub(x[1], x[2]);
        const Cx<T> a = {x[0].x - T(0.5) * t1.x, x[0].y - T(0.5) * t1.y};
        const Cx<T> b = cscale(t2, s3);
        x[0] = cadd(x[0], t1);
        if (!inv) {
            x[1] = cadd(a, mul_mi(b));
            x[2] = cadd(a, mul_pi(b));
        } else {
            x[1] = cadd(a, mul_pi(b));
            x[2] = cadd(a, mul_mi(b));
        }
    }
};

template <typename T>
__device__ __forceinline__ void dft4(Cx<T> &x0, Cx<T> &x1, Cx<T> &x2, Cx<T> &x3, bool inv) {
    const Cx<T> a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
    x0 = cadd(a, c);
    x2 = csub(a, c);
    if (!inv) {
        x1 = cadd(b, mul_mi(d));
        x3 = cadd(b, mul_pi(d));
    } else {
        x1 = cadd(b, mul_pi(d));
        x3 = cadd(b, mul_mi(d));
    }
}

template <typename T>
struct Dft<T, 4> {
    static __device__ __forceinline__ void run(Cx<T> (&x)[4], bool inv, const Cx<T> *, int, int) {
        dft4(x[0], x[1], x[2], x[3], inv);
    }
};

template <typename T>
struct Dft<T, 5> {
    static __device__ __forceinline__ void run(Cx<T> (&x)[5], bool inv, const Cx<T> *, int, int) {
        const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
        const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
        const Cx<T> t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
        const Cx<T> t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
        const Cx<T> a1 = {x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y};
        const Cx<T> a2 = {x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y};
        const Cx<T> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
        const Cx<T> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
        x[0] = cadd(x[0], cadd(t1, t2));
        if (!inv) {
            x[1] = cadd(a1, mul_mi(b1));
            x[4] = cadd(a1, mul_pi(b1));
            x[2] = cadd(a2, mul_mi(b2));
            x[3] = cadd(a2, mul_pi(b2));
        } else {
            x[1] = cadd(a1, mul_pi(b1));
            x[4] = cadd(a1, mul_mi(b1));
            x[2] = cadd(a2, mul_pi(b2));
            x[3] = cadd(a2, mul_mi(b2));
        }
    }
};

template <typename T>
struct Dft<T, 8> {
    static __device__ __forceinline__ void run(Cx<T> (&x)[8], bool inv, const Cx<T> *, int, int) {
        const T h = T(0.70710678118654752440);
        Cx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
        Cx<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
        dft4(e0, e1, e2, e3, inv);
        dft4(o0, o1, o2, o3, inv);
        // o_d *= W8^d, W8 = exp(-+ i pi / 4)
        if (!inv) {
            o1 = {h * (o1.x + o1.y), h * (o1.y - o1.x)};
            o2 = mul_mi(o2);
            o3 = {h * (o3.y - o3.x), -h * (o3.x + o3.y)};
        } else {
            o1 = {h * (o1.x - o1.y), h * (o1.x + o1.y)};
            o2 = mul_pi(o2);
            o3 = {-h * (o3.x + o3.y), h * (o3.x - o3.y)};
        }
        x[0] = cadd(e0, o0);
        x[4] = csub(e0, o0);
        x[1] = cadd(e1, o1);
        x[5] = csub(e1, o1);
        x[2] = cadd(e2, o2);
        x[6] = csub(e2, o2);
        x[3] = cadd(e3, o3);
        x[7] = csub(e3, o3);
    }
};

// One Stockham pass over nb batches stored interleaved: element j of batch b
// at buf[j * nb + b].  Threads take butterflies batch-fastest so that a
// wavefront reads and writes consecutive LDS words.
template <typename T, int R, int PPT>
__device__ __forceinline__ void stockham_pass(Cx<T> *buf, int nb, const FastDiv &nbd, int n,
                                              const PassInfo &ps, const Cx<T> *tw, int tws, bool inv, int tx) {
    constexpr int NT = kFftThreads;
    constexpr int K = (PPT + R - 1) / R;
    const int nbf = nb * (n / R);
    const int m = (int)ps.m.d;
    const int ostride = m * ps.Lstar * nb;
    Cx<T> y[K][R];
    int obase[K];
    #pragma unroll
    for (int k = 0; k < K; ++k) {
        const int t = tx + k * NT;
        obase[k] = -1;
        if (t < nbf) {
            const int w = (int)nbd.div((uint32_t)t);
            const int b = t - w * nb;
            const int p = (int)ps.m.div((uint32_t)w);
            const int q = w - p * m;
            Cx<T> x[R];
            const int ib = (q + m * R * p) * nb + b;
            #pragma unroll
            for (int c = 0; c < R; ++c) x[c] = buf[ib + c * m * nb];
            if (p != 0) {
                #pragma unroll
                for (int c = 1; c < R; ++c) x[c] = cmul(x[c], twid(tw, tws, c * p * m, inv));
            }
            Dft<T, R>::run(x, inv, tw, tws, n);
            #pragma unroll
            for (int d = 0; d < R; ++d) y[k][d] = x[d];
            obase[k] = (q + m * p) * nb + b;
        }
    }
    __syncthreads();
    #pragma unroll
    for (int k = 0; k < K; ++k) {
        if (obase[k] >= 0) {
            #pragma unroll
            for (int d = 0; d < R; ++d) buf[obase[k] + d * ostride] = y[k][d];
        }
    }
    __syncthreads();
}

// Pass with a prime radix R > 13 (known at run time only), each butterfly's
// outputs evaluated directly:
//   y[q + m (p + L* d)] = sum_c w_n^{c m (p + L* d)} x[q + c m + m R p].
// A thread takes B consecutive outputs d0 .. d0 + B - 1 of one butterfly and
// reads each input once: the factor of output d0 + i at term c is
// w_n^{c E0} (w_n^{c n / R})^i with E0 = m (p + L* d0), so per term it reads
// the input and two twiddles from LDS and steps the other B - 1 factors by
// complex multiplication (error growth over at most B - 1 steps).
template <typename T, int PPT>
__device__ __forceinline__ void direct_pass(Cx<T> *buf, int nb, int n, const PassInfo &ps, const Cx<T> *tw, int tws,
                                            bool inv, int tx) {
    constexpr int NT = kFftThreads;
    constexpr int B = 8;
    // work items per thread: items = nb (n / R) ceil(R / B) <= cnt / B + (cnt / R)(B - 1) / B
    // with cnt = nb n <= PPT NT and R >= 17, so at most PPT (17 + B - 1) / (17 B) per thread
    constexpr int KI = (PPT * (17 + B - 1) + 17 * B - 1) / (17 * B);
    const int R = ps.R, m = (int)ps.m.d, Ls = ps.Lstar;
    const int nR = n / R;                       // butterflies per batch (= m L*)
    const int nd = (R + B - 1) / B;             // output blocks per butterfly
    const int items = nb * nR * nd;
    Cx<T> y[KI][B];
    #pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int it = tx + k * NT;
        #pragma unroll
        for (int i = 0; i < B; ++i) y[k][i] = Cx<T>{T(0), T(0)};
        if (it < items) {
            const int b = it % nb;
            const int r1 = it / nb;
            const int db = r1 % nd;
            const int pair = r1 / nd;
            const int q = pair % m;
            const int pp = pair / m;
            const int E0 = m * (pp + Ls * db * B);  // < n
            const int ib = (q + m * R * pp) * nb + b;
            int e0 = 0, es = 0;
            Cx<T> acc[B];
            #pragma unroll
            for (int i = 0; i < B; ++i) acc[i] = Cx<T>{T(0), T(0)};
            for (int c = 0; c < R; ++c) {
                const Cx<T> x = buf[ib + c * m * nb];
                Cx<T> w = twid(tw, tws, e0, inv);
                const Cx<T> st = twid(tw, tws, es, inv);
                #pragma unroll
                for (int i = 0; i < B; ++i) {
                    acc[i] = cadd(acc[i], cmul(x, w));
                    if (i + 1 < B) w = cmul(w, st);
                }
                e0 += E0;
                if (e0 >= n) e0 -= n;
                es += nR;
                if (es >= n) es -= n;
            }
            #pragma unroll
            for (int i = 0; i < B; ++i) y[k][i] = acc[i];
        }
    }
    __syncthreads();
    #pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int it = tx + k * NT;
        if (it < items) {
            const int b = it % nb;
            const int r1 = it / nb;
            const int db = r1 % nd;
            const int pair = r1 / nd;
            const int q = pair % m;
            const int pp = pair / m;
            #pragma unroll
            for (int i = 0; i < B; ++i) {
                const int d = db * B + i;
                if (d < R) buf[(q + m * (pp + Ls * d)) * nb + b] = y[k][i];
            }
        }
    }
    __syncthreads();
}

// GEN = false instantiates only the radices of power-of-two lengths (2, 4, 8),
// which keeps the register footprint of the common case small.
template <typename T, int PPT, bool GEN>
__device__ __forceinline__ void lds_fft(Cx<T> *buf, int nb, const FastDiv &nbd, const AxisFFT &ax,
                                        const Cx<T> *tw, int tws, bool inv, int tx = threadIdx.x) {
    for (int s = 0; s < ax.npass; ++s) {
        const PassInfo &ps = ax.pass[s];
        switch (ps.R) {
        case 2: stockham_pass<T, 2, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
        case 4: stockham_pass<T, 4, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
        case 8: stockham_pass<T, 8, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
        default:
            if constexpr (GEN) {
                switch (ps.R) {
                case 3: stockham_pass<T, 3, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
                case 5: stockham_pass<T, 5, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
                case 7: stockham_pass<T, 7, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
                case 11: stockham_pass<T, 11, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
                case 13: stockham_pass<T, 13, PPT>(buf, nb, nbd, ax.n, ps, tw, tws, inv, tx); break;
                default: direct_pass<T, PPT>(buf, nb, ax.n, ps, tw, tws, inv, tx); break;
                }
            }
            break;
        }
    }
}

template <typename T>
struct FK {
    const T *r;
    const T *q;
    T *r_out;
    Cx<T> *spec;
    const Cx<T> *spec_in;     // middle pass: read from here, write spec (null: in place)
    T *z;
    T *p_upd;                 // fused CG update in the last inverse pass
    T *u_upd;
    double *partial;
    const LcState *st;
    const Cx<T> *tw;          // twiddles of the transformed axis (full length)
    int tws;                  // table stride (2 for the packed last axis)
    const Cx<T> *tw_last;     // last-axis table (post-twiddle of the packed transform)
    const double *om[3];      // e^{2 pi i m / n_a}, interleaved complex
    const double *aa[3];      // (e^{2 pi i m / n_a} - 1) / h_a
    AxisFFT ax;
    FastDiv nbd;              // batches per block
    FastDiv d_nc;             // packed length / FFT length
    FastDiv d_D;              // components
    FastDiv d_nhD;            // nh * D
    FastDiv d_PB;             // pencils per block
    FastDiv d_nh;
    int dim, D, L;
    int n0, n1, nlast, nh;
    long long N, rows, inner_total;
    int RR, PB, nblk, total;
    int lbuf;                 // entries of the LDS tile (last and middle passes): the
                              // dynamic LDS holds the tile, then the twiddle table
    int part_stride;
    int last_even;
    int use_axpy;             // selects the AXPY instantiation on the host
    double out_scale, invN, chalf;  // chalf = element volume / 2
    float near0;              // FP32 plans: sum_a |aa_a|^2 below which M^-1 is formed in FP64
    float hmax_f, post_f;     // FP32 plans: h_max and h_max^2 / chalf (scale-free FP32 inverse)
    T *minv;                  // (B^*B)^-1 table [block][component][slot] (first-axis pass)
    int minv_q;               // 0: slots in order; Q: interleaved for Q-wide loads (see minv_pos)
};

// Position of wavevector slot e in a block's table row.  With q > 0 the
// slots of each run of 64 q are interleaved so that lane l's q-wide vector
// load holds slots l, l + 64, .., l + 64 (q - 1) of the run: a wavefront then
// takes 64 consecutive slots per vector element (consecutive LDS words in the
// first-axis pass) while each lane still loads 16 contiguous bytes.
__host__ __device__ inline int minv_pos(int e, int q) {
    if (q == 0) return e;
    const int run = 64 * q;
    return (e / run) * run + (e % 64) * q + (e % run) / 64;
}

// ---------------------------------------------------------------------------
// Transforms with the shape fixed at compile time: power-of-two length N in
// the plan's default radix order (8 while it divides, then 4 or 2), DS
// sub-problems of NB batches each (NB a power of two), element j of batch b
// of sub-problem s at buf[(s N + j) NB + b].  Every thread index splits into
// (sub-problem, butterfly, batch) by shifts and masks, the LDS offsets of a
// butterfly are compile-time strides and the passes unroll, so the index
// arithmetic that the run-time passes spend in integer multiplies and
// divisions (quarter-rate on this chip) and in bounds branches disappears.
// The butterflies and twiddles are those of stockham_pass, in the same
// order, so the results are the same numbers.
// ---------------------------------------------------------------------------
constexpr int ct_radix_at(int n, int s) {
    int m = n, r = 1;
    for (int i = 0; i <= s; ++i) {
        r = (m % 8 == 0) ? 8 : (m % 4 == 0) ? 4 : 2;
        m /= r;
    }
    return r;
}
constexpr int ct_npass(int n) {
    int k = 0;
    for (int m = n; m > 1; ++k) m /= (m % 8 == 0) ? 8 : (m % 4 == 0) ? 4 : 2;
    return k;
}
constexpr int ct_lstar(int n, int s) {
    int L = 1;
    for (int i = 0; i < s; ++i) L *= ct_radix_at(n, i);
    return L;
}
constexpr int ct_log2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

// Does the run-time schedule of an axis equal the compile-time one of length n?
__host__ inline bool ct_schedule_matches(const AxisFFT &ax, int n) {
    if (ax.n != n || ax.npass != ct_npass(n)) return false;
    for (int s = 0; s < ax.npass; ++s)
        if (ax.pass[s].R != ct_radix_at(n, s)) return false;
    return true;
}

// floor(x / DV) for 0 <= x < RANGE: a shift for powers of two, otherwise
// one full-rate 24-bit multiply by a magic constant and a shift, the
// constant searched and checked over the whole range at compile time.
template <int DV, int RANGE>
struct CtDiv {
    static constexpr bool pow2 = (DV & (DV - 1)) == 0;
    static constexpr bool exact(int sh, unsigned long long m) {
        for (int x = 0; x < RANGE; ++x)
            if ((unsigned long long)x * m >> sh != (unsigned long long)(x / DV)) return false;
        return true;
    }
    static constexpr int find() {
        if (pow2) return ct_log2(DV);
        for (int sh = 0; sh < 32; ++sh) {
            const unsigned long long m = (1ull << sh) / DV + 1;
            if (m < (1ull << 24) && (unsigned long long)(RANGE - 1) * m < (1ull << 32) && exact(sh, m)) return sh;
        }
        return -1;
    }
    static constexpr int SH = find();
    static constexpr unsigned MG = pow2 ? 1u : (unsigned)((1ull << (SH < 0 ? 0 : SH)) / DV + 1);
    static_assert(SH >= 0, "no 24-bit magic divisor for this range");
    static __device__ __forceinline__ int div(int x) {
        if constexpr (pow2) return x >> SH;
        else return (int)(__umul24((unsigned)x, MG) >> SH);
    }
};

// Element j of batch b of sub-problem s sits at buf[(s N + j) NBS + b]; a
// row stride NBS > NB (odd) spreads the lanes of a stride-NBS access over the
// LDS banks.
template <typename T, int N, int NB, int DS, int S, bool INV, int TWS = 1, int NBS = NB>
__device__ __forceinline__ void ct_pass(Cx<T> *buf, const Cx<T> *tw) {
    constexpr int NT = kFftThreads;
    constexpr int R = ct_radix_at(N, S), LS = ct_lstar(N, S);
    constexpr int M = N / (LS * R), BF = N / R;
    constexpr int ITEMS = DS * BF * NB;
    constexpr int K = (ITEMS + NT - 1) / NT;
    constexpr bool EXACT = ITEMS % NT == 0;  // else the last round has idle threads
    constexpr int LBF = ct_log2(BF), LM = ct_log2(M);
    Cx<T> y[K][R];
    int ob[K];
    #pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i0 = threadIdx.x + k * NT;
        const bool on = EXACT || i0 < ITEMS;
        const int i = on ? i0 : 0;
        const int wq = CtDiv<NB, ITEMS>::div(i);  // butterfly index over all sub-problems
        const int b = i - wq * NB;
        const int w = wq & (BF - 1);
        const int sb = (wq >> LBF) * (N * NBS) + b;
        const int p = w >> LM, q = w & (M - 1);
        const int ib = sb + (q + ((p * R) << LM)) * NBS;
        Cx<T> x[R];
        #pragma unroll
        for (int c = 0; c < R; ++c) x[c] = buf[ib + c * M * NBS];
        if constexpr (LS > 1) {
            // butterflies with p = 0 multiply by the twiddle 1 (exact), so
            // the lanes of a wave take no divergent branch
            const int pm = p << LM;
            #pragma unroll
            for (int c = 1; c < R; ++c) x[c] = cmul(x[c], twid(tw, TWS, c * pm, INV));
        }
        Dft<T, R>::run(x, INV, tw, 1, N);
        #pragma unroll
        for (int d = 0; d < R; ++d) y[k][d] = x[d];
        ob[k] = sb + (q + (p << LM)) * NBS;
        if (!on) ob[k] = -1;
    }
    __syncthreads();
    #pragma unroll
    for (int k = 0; k < K; ++k) {
        if (EXACT || ob[k] >= 0) {
            #pragma unroll
            for (int d = 0; d < R; ++d) buf[ob[k] + d * (M * LS * NBS)] = y[k][d];
        }
    }
    __syncthreads();
}

// Passes S .. E - 1 (E = all of them by default).
template <typename T, int N, int NB, int DS, int S, bool INV, int TWS, int NBS, int E = ct_npass(N)>
__device__ __forceinline__ void ct_passes(Cx<T> *buf, const Cx<T> *tw) {
    if constexpr (S < E) {
        ct_pass<T, N, NB, DS, S, INV, TWS, NBS>(buf, tw);
        ct_passes<T, N, NB, DS, S + 1, INV, TWS, NBS, E>(buf, tw);
    }
}

// The whole transform (the buffer already staged and synchronised); the
// twiddle table holds e^{-2 pi i j / (N TWS)} at j (TWS = 2: the table of the
// unpacked length of a packed real transform).
template <typename T, int N, int NB, int DS, bool INV, int TWS = 1, int NBS = NB>
__device__ __forceinline__ void ct_fft(Cx<T> *buf, const Cx<T> *tw) {
    ct_passes<T, N, NB, DS, 0, INV, TWS, NBS>(buf, tw);
}

// Pencils of a compile-time pass per workgroup: N NB points, 16 per thread in
// FP32 (32 KiB of LDS) and 8 in FP64, so that four (FP32) or two (FP64)
// workgroups share a CU.
template <typename T, int N>
constexpr int ct_batches() { return (sizeof(T) == 4 ? 16 : 8) * kFftThreads / N; }

// ---------------------------------------------------------------------------
// last axis, real -> half spectrum (AXPY: fused r -= alpha q, r written back)
//
// Global memory is touched in two phases per kernel: every load of a thread
// is issued before the first use (indices of slots past the end are clamped
// into the block so the loads stay in bounds; their values are discarded),
// then every store; r and r_out may be the same buffer.
// ---------------------------------------------------------------------------
template <typename T, int PPT, bool GEN, bool AXPY>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(kGenWaves<T, GEN>))) void k_last_fwd(FK<T> a) {
    constexpr int NT = kFftThreads;
    __shared__ Cx<T> sbuf[GEN ? 1 : PPT * NT];
    Cx<T> *buf = GEN ? reinterpret_cast<Cx<T> *>(feh_dyn_lds) : sbuf;
    int t = xcd_remap(blockIdx.x, a.total);
    const int lc = t / a.nblk;
    const int blk = t - lc * a.nblk;
    T alpha = T(0);
    if (a.st) {
        if (!a.st[lc].active) return;
        if (AXPY) alpha = T(a.st[lc].alpha);
    }
    const int D = a.D;
    const int nb = D * a.RR;
    const long long s0 = (long long)blk * a.RR;
    const int nrows = (int)min((long long)a.RR, a.rows - s0);
    const int nc = a.ax.n;
    const int cnt = nb * nc;
    const long long N = a.N;
    const int even = a.last_even;
    Cx<T> *twl = GEN ? buf + a.lbuf : reinterpret_cast<Cx<T> *>(feh_dyn_lds);
    stage(twl, a.tw_last, a.nlast);
    const long long lbase = (long long)lc * D * N + s0 * a.nlast;
    // AXPY keeps two loads per slot in flight: 8 slots per round
    constexpr int CH = AXPY ? 8 : PPT;
    #pragma unroll
    for (int h = 0; h < PPT; h += CH) {
        Cx<T> v[CH];
        Cx<T> w[AXPY ? CH : 1];
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e0 = threadIdx.x + (h + k) * NT;
            const int e = e0 < cnt ? e0 : 0;
            const int b = (int)a.d_nc.div((uint32_t)e);
            const int j = e - b * nc;
            const int sl0 = (int)a.d_D.div((uint32_t)b);
            const int c = b - sl0 * D;
            const int sl = sl0 < nrows ? sl0 : nrows - 1;
            // element offset of the packed pair (even) or of the sample (odd)
            const long long off = lbase + (long long)c * N + (long long)sl * a.nlast + (even ? 2 * j : j);
            if (even) {
                v[k] = *reinterpret_cast<const Cx<T> *>(a.r + off);
                if (AXPY) w[k] = *reinterpret_cast<const Cx<T> *>(a.q + off);
            } else {
                v[k] = Cx<T>{a.r[off], T(0)};
                if (AXPY) w[k] = Cx<T>{a.q[off], T(0)};
            }
        }
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e0 = threadIdx.x + (h + k) * NT;
            const int e = e0 < cnt ? e0 : 0;
            const int b = (int)a.d_nc.div((uint32_t)e);
            const int j = e - b * nc;
            const int sl = (int)a.d_D.div((uint32_t)b);
            const int c = b - sl * D;
            const bool ok = e0 < cnt && sl < nrows;
            if (AXPY) {
                v[k].x -= alpha * w[k].x;
                v[k].y -= alpha * w[k].y;
                if (ok) {
                    const long long off = lbase + (long long)c * N + (long long)sl * a.nlast + (even ? 2 * j : j);
                    if (even) *reinterpret_cast<Cx<T> *>(a.r_out + off) = v[k];
                    else a.r_out[off] = v[k].x;
                }
            }
            if (!ok) v[k] = Cx<T>{T(0), T(0)};
            if (e0 < cnt) buf[j * nb + b] = v[k];
        }
    }
    __syncthreads();
    lds_fft<T, PPT, GEN>(buf, nb, a.nbd, a.ax, twl, a.tws, false);
    // untangle the packed transform and store the half spectrum, components
    // fastest; the count nrows * nh * D exceeds PPT * NT by at most nb
    const int nh = a.nh;
    const int ocnt = nrows * nh * D;
    Cx<T> X[PPT + 1];
    #pragma unroll
    for (int k = 0; k < PPT + 1; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int e = e0 < ocnt ? e0 : 0;
        const int kk = (int)a.d_D.div((uint32_t)e);
        const int c = e - kk * D;
        const int sl = (int)a.d_nh.div((uint32_t)kk);
        const int kx = kk - sl * nh;
        const int b = sl * D + c;
        if (even) {
            const int ka = (kx == nc) ? 0 : kx;
            const int kb = (kx == 0) ? 0 : nc - kx;
            const Cx<T> Zk = buf[ka * nb + b], Zm = cconj(buf[kb * nb + b]);
            const Cx<T> A = {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y + Zm.y)};
            const Cx<T> dZ = csub(Zk, Zm);
            const Cx<T> B = {T(0.5) * dZ.y, -T(0.5) * dZ.x};  // -i/2 (Zk - conj Z(nc-k))
            X[k] = cadd(A, cmul(twl[kx], B));
        } else {
            X[k] = buf[kx * nb + b];
        }
    }
    Cx<T> *dst = a.spec + ((long long)lc * a.rows + s0) * (long long)nh * D;
    #pragma unroll
    for (int k = 0; k < PPT + 1; ++k) {
        const int e0 = threadIdx.x + k * NT;
        if (e0 < ocnt) dst[e0] = X[k];
    }
}

// ---------------------------------------------------------------------------
// last axis, half spectrum -> real (times out_scale).  UPD: the real result z
// is not stored; instead the CG update u += alpha_pend p, p = z + beta p is
// applied in place (one pass over p and u while z is in registers).
// ---------------------------------------------------------------------------
template <typename T, int PPT, bool GEN, bool UPD>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(kGenWaves<T, GEN>))) void k_last_inv(FK<T> a) {
    constexpr int NT = kFftThreads;
    __shared__ Cx<T> sbuf[GEN ? 1 : PPT * NT];
    Cx<T> *buf = GEN ? reinterpret_cast<Cx<T> *>(feh_dyn_lds) : sbuf;
    int t = xcd_remap(blockIdx.x, a.total);
    const int lc = t / a.nblk;
    const int blk = t - lc * a.nblk;
    if (a.st && !a.st[lc].active) return;
    const int D = a.D;
    const int nb = D * a.RR;
    const long long s0 = (long long)blk * a.RR;
    const int nrows = (int)min((long long)a.RR, a.rows - s0);
    const int nc = a.ax.n;
    const int nh = a.nh;
    const int cnt = nb * nc;
    const long long N = a.N;
    const int even = a.last_even;
    Cx<T> *twl = GEN ? buf + a.lbuf : reinterpret_cast<Cx<T> *>(feh_dyn_lds);
    stage(twl, a.tw_last, a.nlast);
    __syncthreads();
    // gather e -> (sl, k, c), components fastest (coalesced spectrum reads);
    // the packed input Z(k) needs X(k) and X(nc - k)
    const Cx<T> *src = a.spec + ((long long)lc * a.rows + s0) * (long long)nh * D;
    constexpr int CH = PPT / 2;
    #pragma unroll
    for (int h = 0; h < PPT; h += CH) {
        Cx<T> Xa[CH], Xb[CH];
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e0 = threadIdx.x + (h + k) * NT;
            const int e = e0 < cnt ? e0 : 0;
            const int kk = (int)a.d_D.div((uint32_t)e);
            const int c = e - kk * D;
            const int sl0 = (int)a.d_nc.div((uint32_t)kk);
            const int kx = kk - sl0 * nc;
            const int sl = sl0 < nrows ? sl0 : nrows - 1;
            const Cx<T> *row = src + (long long)sl * nh * D + c;
            if (even) {
                Xa[k] = row[(long long)kx * D];
                Xb[k] = row[(long long)(nc - kx) * D];
            } else {
                Xa[k] = row[(long long)(kx < nh ? kx : a.nlast - kx) * D];
            }
        }
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e0 = threadIdx.x + (h + k) * NT;
            const int e = e0 < cnt ? e0 : 0;
            const int kk = (int)a.d_D.div((uint32_t)e);
            const int c = e - kk * D;
            const int sl = (int)a.d_nc.div((uint32_t)kk);
            const int kx = kk - sl * nc;
            // the DC and Nyquist samples of a real signal's spectrum are real:
            // their imaginary parts (rounding residue) are dropped
            if (kx == 0) {
                Xa[k].y = T(0);
                Xb[k].y = T(0);
            }
            Cx<T> Z;
            if (even) {
                const Cx<T> Xm = cconj(Xb[k]);
                const Cx<T> A = cadd(Xa[k], Xm);
                const Cx<T> B = cmulc(csub(Xa[k], Xm), twl[kx]);  // exp(+2 pi i k / n) (Xk - conj X(nc-k))
                Z = cadd(A, mul_pi(B));
            } else {
                Z = kx < nh ? Xa[k] : cconj(Xa[k]);
            }
            if (sl >= nrows) Z = Cx<T>{T(0), T(0)};
            if (e0 < cnt) buf[kx * nb + sl * D + c] = Z;
        }
    }
    __syncthreads();
    lds_fft<T, PPT, GEN>(buf, nb, a.nbd, a.ax, twl, a.tws, true);
    const T sc = T(a.out_scale);
    Cx<T> y[PPT];
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int e = e0 < cnt ? e0 : 0;
        const int b = (int)a.d_nc.div((uint32_t)e);
        const int j = e - b * nc;
        y[k] = buf[j * nb + b];
    }
    const long long lbase = (long long)lc * D * N + s0 * a.nlast;
    if constexpr (UPD) {
        const T beta = T(a.st[lc].beta), ap = T(a.st[lc].alpha_pend);
        constexpr int CH = 8;  // slots per round: two loads each in flight
        #pragma unroll
        for (int h = 0; h < PPT; h += CH) {
            Cx<T> pv[CH], uv[CH];
            #pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e0 = threadIdx.x + (h + k) * NT;
                const int e = e0 < cnt ? e0 : 0;
                const int b = (int)a.d_nc.div((uint32_t)e);
                const int j = e - b * nc;
                const int sl0 = (int)a.d_D.div((uint32_t)b);
                const int c = b - sl0 * D;
                const int sl = sl0 < nrows ? sl0 : nrows - 1;
                const long long o = lbase + (long long)c * N + (long long)sl * a.nlast + (even ? 2 * j : j);
                if (even) {
                    pv[k] = ldc_nt(reinterpret_cast<const Cx<T> *>(a.p_upd + o));
                    uv[k] = ldc_nt(reinterpret_cast<const Cx<T> *>(a.u_upd + o));
                } else {
                    pv[k] = Cx<T>{ldr_nt(a.p_upd + o), T(0)};
                    uv[k] = Cx<T>{ldr_nt(a.u_upd + o), T(0)};
                }
            }
            #pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int e0 = threadIdx.x + (h + k) * NT;
                const int b = (int)a.d_nc.div((uint32_t)e0);
                const int j = e0 - b * nc;
                const int sl = (int)a.d_D.div((uint32_t)b);
                const int c = b - sl * D;
                if (e0 < cnt && sl < nrows) {
                    const long long o = lbase + (long long)c * N + (long long)sl * a.nlast + (even ? 2 * j : j);
                    const Cx<T> z = {y[h + k].x * sc, y[h + k].y * sc};
                    const Cx<T> un = {uv[k].x + ap * pv[k].x, uv[k].y + ap * pv[k].y};
                    const Cx<T> pn = {z.x + beta * pv[k].x, z.y + beta * pv[k].y};
                    if (even) {
                        stc_nt(reinterpret_cast<Cx<T> *>(a.u_upd + o), un);
                        stc_nt(reinterpret_cast<Cx<T> *>(a.p_upd + o), pn);
                    } else {
                        str_nt(a.u_upd + o, un.x);
                        str_nt(a.p_upd + o, pn.x);
                    }
                }
            }
        }
    } else {
        #pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e0 = threadIdx.x + k * NT;
            const int b = (int)a.d_nc.div((uint32_t)e0);
            const int j = e0 - b * nc;
            const int sl = (int)a.d_D.div((uint32_t)b);
            const int c = b - sl * D;
            if (e0 < cnt && sl < nrows) {
                const long long o = lbase + (long long)c * N + (long long)sl * a.nlast;
                if (even) stc_nt(reinterpret_cast<Cx<T> *>(a.z + o) + j, Cx<T>{y[k].x * sc, y[k].y * sc});
                else str_nt(a.z + o + j, y[k].x * sc);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Last-axis passes with the compile-time transform: even length NL (packed
// into NC = NL / 2 complex points) in the default radix order, RR rows of D
// components per workgroup (24 points per thread in FP32), the LDS tile and
// the global layouts of k_last_fwd / k_last_inv (batch b = row D + component,
// element j at buf[j NBS + b], NBS = ct_last_stride).  Same arithmetic in the
// same order.
// ---------------------------------------------------------------------------
template <int NL, int D>
constexpr int ct_last_rows() { return 24 * kFftThreads / (NL / 2 * D); }
// LDS row stride of the tile: one past the D RR batches (odd, so that the
// transposing accesses, consecutive lanes one row apart, hit distinct banks)
// when three workgroups still fit a CU's LDS with it, else D RR
template <int NL, int D>
constexpr int ct_last_stride() {
    constexpr int NB = D * ct_last_rows<NL, D>();
    return (NB + 1) * (NL / 2) * 8 + NL * 8 <= 160 * 1024 / 3 ? NB + 1 : NB;
}

// Byte offset of packed pair j of row sl (of the block) and component c in
// the load case's real SoA field [D][N].
template <typename T, int NL, int D>
__device__ __forceinline__ unsigned last_pair_offset(int c, int sl, int j, unsigned N32, unsigned row0) {
    // c N: N is a multiple of NL >= 128, so one 24-bit multiply of N / 128
    static_assert(NL % 128 == 0, "component stride from N / 128");
    const unsigned cb = __umul24((unsigned)c, N32 >> 7) << 7;
    return (cb + row0 + (unsigned)(sl * NL + 2 * j)) * (unsigned)sizeof(T);
}

// MODE 0: r -> half spectrum; MODE 1 (AXPY): r -= alpha q, r written back, its
// half spectrum written; MODE 2 (RSPEC): the half spectrum of q, and the
// residual kept as a half spectrum updated in place, spec -= alpha q^.
template <typename T, int NL, int D, int MODE, bool FULL>
__device__ __forceinline__ void last_fwd_ct_body(const FK<T> &a, int lc, long long s0, int nrows, T alpha,
                                                 Cx<T> *buf, const Cx<T> *twl) {
    constexpr int NT = kFftThreads, NC = NL / 2, NH = NC + 1;
    constexpr int RR = ct_last_rows<NL, D>(), NB = D * RR, NBS = ct_last_stride<NL, D>();
    constexpr int CNT = NB * NC, PPT = CNT / NT;
    constexpr int OCNT = RR * NH * D;                  // half-spectrum values of the block
    constexpr int KO = (OCNT + NT - 1) / NT;
    constexpr int LNC = ct_log2(NC);
    const long long lbase = (long long)lc * D * a.N;
    constexpr bool AXPY = MODE == 1;
    const T *rl = MODE == 2 ? a.q + lbase : a.r + lbase;  // the transformed field
    const T *ql = AXPY ? a.q + lbase : nullptr;
    T *rol = AXPY ? a.r_out + lbase : nullptr;
    const unsigned N32 = (unsigned)a.N, row0 = (unsigned)(s0 * NL);
    // slot e -> batch b = e / NC (row sl = b / D, component c), packed pair j
    constexpr int CH = AXPY ? 8 : PPT;
    #pragma unroll
    for (int h = 0; h < PPT; h += CH) {
        Cx<T> v[CH];
        Cx<T> w[AXPY ? CH : 1];
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = threadIdx.x + (h + k) * NT;
            const int b = e >> LNC, j = e & (NC - 1);
            const int sl0 = CtDiv<D, NB>::div(b), c = b - sl0 * D;
            const int sl = (FULL || sl0 < nrows) ? sl0 : nrows - 1;
            const unsigned off = last_pair_offset<T, NL, D>(c, sl, j, N32, row0);
            v[k] = *at_byte(reinterpret_cast<const Cx<T> *>(rl), off);
            if (AXPY) w[k] = *at_byte(reinterpret_cast<const Cx<T> *>(ql), off);
        }
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = threadIdx.x + (h + k) * NT;
            const int b = e >> LNC, j = e & (NC - 1);
            const int sl = CtDiv<D, NB>::div(b), c = b - sl * D;
            const bool ok = FULL || sl < nrows;
            if (AXPY) {
                v[k].x -= alpha * w[k].x;
                v[k].y -= alpha * w[k].y;
                if (ok) *at_byte(reinterpret_cast<Cx<T> *>(rol), last_pair_offset<T, NL, D>(c, sl, j, N32, row0)) = v[k];
            }
            buf[j * NBS + b] = ok ? v[k] : Cx<T>{T(0), T(0)};
        }
    }
    __syncthreads();
    ct_fft<T, NC, NB, 1, false, 2, NBS>(buf, twl);
    // untangle the packed transform; half spectrum out, components fastest
    Cx<T> X[KO];
    #pragma unroll
    for (int k = 0; k < KO; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int e = (OCNT % NT == 0 || e0 < OCNT) ? e0 : 0;
        const int kk = CtDiv<D, OCNT>::div(e);
        const int c = e - kk * D;
        const int sl = CtDiv<NH, OCNT / D>::div(kk);
        const int kx = kk - sl * NH;
        const int b = sl * D + c;
        const int ka = (kx == NC) ? 0 : kx;
        const int kb = (kx == 0) ? 0 : NC - kx;
        const Cx<T> Zk = buf[ka * NBS + b], Zm = cconj(buf[kb * NBS + b]);
        const Cx<T> A = {T(0.5) * (Zk.x + Zm.x), T(0.5) * (Zk.y + Zm.y)};
        const Cx<T> dZ = csub(Zk, Zm);
        const Cx<T> B = {T(0.5) * dZ.y, -T(0.5) * dZ.x};  // -i/2 (Zk - conj Z(nc-k))
        X[k] = cadd(A, cmul(twl[kx], B));
    }
    Cx<T> *dst = a.spec + ((long long)lc * a.rows + s0) * (long long)NH * D;
    const int ocnt = FULL ? OCNT : nrows * NH * D;
    if constexpr (MODE == 2) {
        // every load before the first store
        Cx<T> R[KO];
        #pragma unroll
        for (int k = 0; k < KO; ++k) {
            const int e0 = threadIdx.x + k * NT;
            const int e = ((FULL && (OCNT % NT == 0 || k + 1 < KO)) || e0 < ocnt) ? e0 : 0;
            R[k] = *at_byte(dst, (unsigned)e * (unsigned)sizeof(Cx<T>));
        }
        #pragma unroll
        for (int k = 0; k < KO; ++k) {
            const int e0 = threadIdx.x + k * NT;
            if ((FULL && (OCNT % NT == 0 || k + 1 < KO)) || e0 < ocnt)
                *at_byte(dst, (unsigned)e0 * (unsigned)sizeof(Cx<T>)) =
                    Cx<T>{R[k].x - alpha * X[k].x, R[k].y - alpha * X[k].y};
        }
    } else {
        #pragma unroll
        for (int k = 0; k < KO; ++k) {
            const int e0 = threadIdx.x + k * NT;
            if ((FULL && (OCNT % NT == 0 || k + 1 < KO)) || e0 < ocnt) *at_byte(dst, (unsigned)e0 * (unsigned)sizeof(Cx<T>)) = X[k];
        }
    }
}

template <typename T, int NL, int D, int MODE>
__global__ __launch_bounds__(kFftThreads) void k_last_fwd_ct(FK<T> a) {
    constexpr int NT = kFftThreads, NC = NL / 2;
    constexpr int RR = ct_last_rows<NL, D>(), NB = D * RR;
    static_assert((NB * NC) % NT == 0, "whole slots per thread");
    __shared__ Cx<T> buf[ct_last_stride<NL, D>() * NC];
    __shared__ Cx<T> twl[NL];
    const int t = xcd_remap(blockIdx.x, a.total);
    const int lc = t / a.nblk;
    const int blk = t - lc * a.nblk;
    T alpha = T(0);
    if (a.st) {
        if (!a.st[lc].active) return;
        if (MODE != 0) alpha = T(a.st[lc].alpha);
    }
    const long long s0 = (long long)blk * RR;
    const int nrows = (int)min((long long)RR, a.rows - s0);
    for (int i = threadIdx.x; i < NL; i += NT) twl[i] = a.tw_last[i];
    if (nrows == RR) last_fwd_ct_body<T, NL, D, MODE, true>(a, lc, s0, nrows, alpha, buf, twl);
    else last_fwd_ct_body<T, NL, D, MODE, false>(a, lc, s0, nrows, alpha, buf, twl);
}

template <typename T, int NL, int D, bool UPD, bool FULL>
__device__ __forceinline__ void last_inv_ct_body(const FK<T> &a, int lc, long long s0, int nrows, Cx<T> *buf,
                                                 const Cx<T> *twl) {
    constexpr int NT = kFftThreads, NC = NL / 2, NH = NC + 1;
    constexpr int RR = ct_last_rows<NL, D>(), NB = D * RR, NBS = ct_last_stride<NL, D>();
    constexpr int CNT = NB * NC, PPT = CNT / NT;
    constexpr int LNC = ct_log2(NC);
    // gather e -> (row sl, k, component c), components fastest; the packed
    // input Z(k) needs X(k) and X(nc - k)
    const Cx<T> *src = a.spec + ((long long)lc * a.rows + s0) * (long long)NH * D;
    constexpr int CH = PPT / 2;
    #pragma unroll
    for (int h = 0; h < PPT; h += CH) {
        Cx<T> Xa[CH], Xb[CH];
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = threadIdx.x + (h + k) * NT;
            const int kk = CtDiv<D, CNT>::div(e);
            const int c = e - kk * D;
            const int sl0 = kk >> LNC, kx = kk & (NC - 1);
            const int sl = (FULL || sl0 < nrows) ? sl0 : nrows - 1;
            const unsigned row = (unsigned)(sl * (NH * D) + c);
            Xa[k] = *at_byte(src, (row + (unsigned)(kx * D)) * (unsigned)sizeof(Cx<T>));
            Xb[k] = *at_byte(src, (row + (unsigned)((NC - kx) * D)) * (unsigned)sizeof(Cx<T>));
        }
        #pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int e = threadIdx.x + (h + k) * NT;
            const int kk = CtDiv<D, CNT>::div(e);
            const int c = e - kk * D;
            const int sl = kk >> LNC, kx = kk & (NC - 1);
            // the DC and Nyquist samples of a real signal's spectrum are real:
            // their imaginary parts (rounding residue) are dropped
            const Cx<T> xa = {Xa[k].x, kx == 0 ? T(0) : Xa[k].y};
            const Cx<T> Xm = {Xb[k].x, kx == 0 ? T(0) : -Xb[k].y};
            const Cx<T> A = cadd(xa, Xm);
            const Cx<T> B = cmulc(csub(xa, Xm), twl[kx]);  // exp(+2 pi i k / n) (Xk - conj X(nc-k))
            Cx<T> Z = cadd(A, mul_pi(B));
            if (!FULL && sl >= nrows) Z = Cx<T>{T(0), T(0)};
            buf[kx * NBS + sl * D + c] = Z;
        }
    }
    __syncthreads();
    ct_fft<T, NC, NB, 1, true, 2, NBS>(buf, twl);
    const T sc = T(a.out_scale);
    Cx<T> y[PPT];
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int b = e >> LNC, j = e & (NC - 1);
        y[k] = buf[j * NBS + b];
    }
    const long long lbase = (long long)lc * D * a.N;
    const unsigned N32 = (unsigned)a.N, row0 = (unsigned)(s0 * NL);
    if constexpr (UPD) {
        Cx<T> *pl = reinterpret_cast<Cx<T> *>(a.p_upd + lbase);
        Cx<T> *ul = reinterpret_cast<Cx<T> *>(a.u_upd + lbase);
        const T beta = T(a.st[lc].beta), ap = T(a.st[lc].alpha_pend);
        constexpr int CH2 = 8;  // slots per round: two loads each in flight
        #pragma unroll
        for (int h = 0; h < PPT; h += CH2) {
            Cx<T> pv[CH2], uv[CH2];
            #pragma unroll
            for (int k = 0; k < CH2; ++k) {
                const int e = threadIdx.x + (h + k) * NT;
                const int b = e >> LNC, j = e & (NC - 1);
                const int sl0 = CtDiv<D, NB>::div(b), c = b - sl0 * D;
                const int sl = (FULL || sl0 < nrows) ? sl0 : nrows - 1;
                const unsigned o = last_pair_offset<T, NL, D>(c, sl, j, N32, row0);
                pv[k] = ldc_nt(at_byte(pl, o));
                uv[k] = ldc_nt(at_byte(ul, o));
            }
            #pragma unroll
            for (int k = 0; k < CH2; ++k) {
                const int e = threadIdx.x + (h + k) * NT;
                const int b = e >> LNC, j = e & (NC - 1);
                const int sl = CtDiv<D, NB>::div(b), c = b - sl * D;
                if (FULL || sl < nrows) {
                    const unsigned o = last_pair_offset<T, NL, D>(c, sl, j, N32, row0);
                    const Cx<T> z = {y[h + k].x * sc, y[h + k].y * sc};
                    const Cx<T> un = {uv[k].x + ap * pv[k].x, uv[k].y + ap * pv[k].y};
                    const Cx<T> pn = {z.x + beta * pv[k].x, z.y + beta * pv[k].y};
                    stc_nt(at_byte(ul, o), un);
                    stc_nt(at_byte(pl, o), pn);
                }
            }
        }
    } else {
        Cx<T> *zl = reinterpret_cast<Cx<T> *>(a.z + lbase);
        #pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int e = threadIdx.x + k * NT;
            const int b = e >> LNC, j = e & (NC - 1);
            const int sl = CtDiv<D, NB>::div(b), c = b - sl * D;
            if (FULL || sl < nrows)
                stc_nt(at_byte(zl, last_pair_offset<T, NL, D>(c, sl, j, N32, row0)), Cx<T>{y[k].x * sc, y[k].y * sc});
        }
    }
}

template <typename T, int NL, int D, bool UPD>
__global__ __launch_bounds__(kFftThreads) void k_last_inv_ct(FK<T> a) {
    constexpr int NT = kFftThreads, NC = NL / 2;
    constexpr int RR = ct_last_rows<NL, D>(), NB = D * RR;
    static_assert((NB * NC) % NT == 0, "whole slots per thread");
    __shared__ Cx<T> buf[ct_last_stride<NL, D>() * NC];
    __shared__ Cx<T> twl[NL];
    const int t = xcd_remap(blockIdx.x, a.total);
    const int lc = t / a.nblk;
    const int blk = t - lc * a.nblk;
    if (a.st && !a.st[lc].active) return;
    const long long s0 = (long long)blk * RR;
    const int nrows = (int)min((long long)RR, a.rows - s0);
    for (int i = threadIdx.x; i < NL; i += NT) twl[i] = a.tw_last[i];
    __syncthreads();
    if (nrows == RR) last_inv_ct_body<T, NL, D, UPD, true>(a, lc, s0, nrows, buf, twl);
    else last_inv_ct_body<T, NL, D, UPD, false>(a, lc, s0, nrows, buf, twl);
}

// ---------------------------------------------------------------------------
// middle axis (3D), complex to complex
// ---------------------------------------------------------------------------
template <typename T, int PPT, bool GEN>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(kGenWaves<T, GEN>))) void k_middle(FK<T> a, int inv) {
    constexpr int NT = kFftThreads;
    __shared__ Cx<T> sbuf[GEN ? 1 : PPT * NT];
    Cx<T> *buf = GEN ? reinterpret_cast<Cx<T> *>(feh_dyn_lds) : sbuf;
    int t = xcd_remap(blockIdx.x, a.total);
    const int ib = t % a.nblk;
    t /= a.nblk;
    const int i0 = t % a.n0;
    const int lc = t / a.n0;
    if (a.st && !a.st[lc].active) return;
    const int PB = a.PB;
    const int n1 = a.n1;
    const int cnt = PB * n1;
    const long long inner = a.inner_total;
    const long long in0 = (long long)ib * PB;
    const long long boff = ((long long)lc * a.n0 + i0) * n1 * inner + in0;
    Cx<T> *base = a.spec + boff;
    const Cx<T> *src = (a.spec_in ? a.spec_in : a.spec) + boff;
    const int lim = (int)min((long long)PB, inner - in0);
    Cx<T> *twl = GEN ? buf + a.lbuf : reinterpret_cast<Cx<T> *>(feh_dyn_lds);
    stage(twl, a.tw, n1);
    Cx<T> v[PPT];
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int e = e0 < cnt ? e0 : 0;
        const int j = (int)a.d_PB.div((uint32_t)e);
        const int b = e - j * PB;
        v[k] = src[(long long)j * inner + (b < lim ? b : lim - 1)];
    }
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int j = (int)a.d_PB.div((uint32_t)e0);
        const int b = e0 - j * PB;
        if (e0 < cnt) buf[e0] = (b < lim) ? v[k] : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    lds_fft<T, PPT, GEN>(buf, PB, a.d_PB, a.ax, twl, 1, inv != 0);
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e0 = threadIdx.x + k * NT;
        v[k] = buf[e0 < cnt ? e0 : 0];
    }
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e0 = threadIdx.x + k * NT;
        const int j = (int)a.d_PB.div((uint32_t)e0);
        const int b = e0 - j * PB;
        if (e0 < cnt && b < lim) base[(long long)j * inner + b] = v[k];
    }
}

// Middle axis with the compile-time transform of length N (= n1): the
// workgroup takes NB consecutive (kh, component) pencils of one (load case,
// axis-0 index), as k_middle does with its run-time pencil count.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kFftThreads) void k_middle_ct(FK<T> a) {
    constexpr int NT = kFftThreads;
    constexpr int NB = ct_batches<T, N>();
    constexpr int PPT = N * NB / NT;
    constexpr int LNB = ct_log2(NB);
    __shared__ Cx<T> buf[N * NB];
    __shared__ Cx<T> twl[N];
    int t = xcd_remap(blockIdx.x, a.total);
    const int ib = t % a.nblk;
    t /= a.nblk;
    const int i0 = t % a.n0;
    const int lc = t / a.n0;
    if (a.st && !a.st[lc].active) return;
    const unsigned inner = (unsigned)a.inner_total;
    const unsigned in0 = (unsigned)ib * NB;
    const long long boff = ((long long)lc * a.n0 + i0) * (long long)N * inner + in0;
    Cx<T> *base = a.spec + boff;
    const Cx<T> *src = (a.spec_in ? a.spec_in : a.spec) + boff;
    const int lim = min(NB, (int)(inner - in0));
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = a.tw[i];
    Cx<T> v[PPT];
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int j = e >> LNB, b = e & (NB - 1);
        v[k] = src[__umul24((unsigned)j, inner) + (unsigned)(b < lim ? b : lim - 1)];
    }
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = threadIdx.x + k * NT;
        buf[e] = ((e & (NB - 1)) < lim) ? v[k] : Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    ct_fft<T, N, NB, 1, INV>(buf, twl);
    #pragma unroll
    for (int k = 0; k < PPT; ++k) v[k] = buf[threadIdx.x + k * NT];
    #pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int j = e >> LNB, b = e & (NB - 1);
        if (b < lim) base[__umul24((unsigned)j, inner) + (unsigned)b] = v[k];
    }
}

// ---------------------------------------------------------------------------
// first axis: forward, per-wavevector (B^*B)^-1 solve with Parseval r.z,
// inverse (mode 0); forward only (mode 1); inverse only (mode 2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ Cx<double> ld2(const double *p, int i) { return Cx<double>{p[2 * i], p[2 * i + 1]}; }
template <typename R>
__device__ __forceinline__ R nrm(Cx<R> a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Inverse of the Hermitian positive definite M (diagonal Md, upper triangle
// Mo = (M01, M02, M12)) by the adjugate in the scalar type R: Id = real
// diagonal, Io = upper triangle of post M^-1.
template <typename R, int D>
__device__ __forceinline__ void herm_inverse(const R (&Md)[D], const Cx<R> (&Mo)[3], R (&Id)[D], Cx<R> (&Io)[3],
                                             R post = R(1)) {
    if constexpr (D == 2) {
        const R id = post * recip(Md[0] * Md[1] - nrm(Mo[0]));
        Id[0] = Md[1] * id;
        Id[1] = Md[0] * id;
        Io[0] = cscale(Mo[0], -id);
        Io[1] = Io[2] = Cx<R>{R(0), R(0)};
    } else {
        const Cx<R> a = Mo[0], b = Mo[1], c = Mo[2];
        const R C0 = Md[1] * Md[2] - nrm(c);
        const R C1 = Md[0] * Md[2] - nrm(b);
        const R C2 = Md[0] * Md[1] - nrm(a);
        const Cx<R> A01 = csub(cmulc(b, c), cscale(a, Md[2]));  // b conj(c) - a d2
        const Cx<R> A02 = csub(cmul(a, c), cscale(b, Md[1]));   // a c - b d1
        const Cx<R> A12 = csub(cmulc(b, a), cscale(c, Md[0]));  // b conj(a) - c d0
        // det = d0 C00 + Re(a conj(A01)) + Re(b conj(A02))
        const R det = Md[0] * C0 + (a.x * A01.x + a.y * A01.y) + (b.x * A02.x + b.y * A02.y);
        const R id = post * recip(det);
        Id[0] = C0 * id;
        Id[1] = C1 * id;
        Id[2] = C2 * id;
        Io[0] = cscale(A01, id);
        Io[1] = cscale(A02, id);
        Io[2] = cscale(A12, id);
    }
}

// M(k) = B^*B(k) of the linear elements of one voxel (six Kuhn tetrahedra in
// 3D, two triangles in 2D) from the per-axis factors aa_a = (w_a - 1) / h_a
// and w_a = e^{2 pi i m_a / n_a}, in the scalar type R; ch = element volume / 2.
template <typename R, int DIM>
__device__ __forceinline__ void core_matrix(const Cx<R> (&aa)[3], const Cx<R> (&w)[3], R ch, R (&Md)[DIM],
                                            Cx<R> (&Mo)[3]) {
    if constexpr (DIM == 3) {
        const Cx<R> a0 = aa[0], a1 = aa[1], a2 = aa[2];
        const Cx<R> w0 = w[0], w1 = w[1], w2 = w[2];
        const R n0s = nrm(a0), n1s = nrm(a1), n2s = nrm(a2);
        const R S = R(6) * (n0s + n1s + n2s);
        Md[0] = ch * (S + R(6) * n0s);
        Md[1] = ch * (S + R(6) * n1s);
        Md[2] = ch * (S + R(6) * n2s);
        const Cx<R> two = {R(2), R(0)};
        // M_ab = ch a_a conj(a_b) [conj(w_a)(2 + conj(w_c)) + w_b (2 + w_c)]
        Mo[0] = cscale(cmul(cmulc(a0, a1), cadd(cmulc(cadd(two, cconj(w2)), w0), cmul(w1, cadd(two, w2)))), ch);
        Mo[1] = cscale(cmul(cmulc(a0, a2), cadd(cmulc(cadd(two, cconj(w1)), w0), cmul(w2, cadd(two, w1)))), ch);
        Mo[2] = cscale(cmul(cmulc(a1, a2), cadd(cmulc(cadd(two, cconj(w0)), w1), cmul(w2, cadd(two, w0)))), ch);
    } else {
        const Cx<R> a0 = aa[0], a1 = aa[1];
        const Cx<R> w0 = w[0], w1 = w[1];
        const R n0s = nrm(a0), n1s = nrm(a1);
        const R S = R(2) * (n0s + n1s);
        Md[0] = ch * (S + R(2) * n0s);
        Md[1] = ch * (S + R(2) * n1s);
        // M_01 = ch a0 conj(a1) (1 + w1 conj(w0))
        const Cx<R> f = {R(1) + (w1.x * w0.x + w1.y * w0.y), w1.y * w0.x - w1.x * w0.y};
        Mo[0] = cscale(cmul(cmulc(a0, a1), f), ch);
        Mo[1] = Mo[2] = Cx<R>{R(0), R(0)};
    }
}

// Inverse of the projection core at wavevector slot e of the workgroup, in
// the plan precision: md = real diagonal, mo = upper triangle of M(k)^-1 (zero
// at k = 0 and for slots past the block's pencils); the Parseval weight bit of
// the slot.  The per-axis factors come from FP64 tables.  FP64 plans form the
// inverse in FP64.  FP32 plans form it in FP32 where sum_a |aa_a|^2 >= near0
// and in FP64 (rounded once) at the long-wavelength wavevectors below it,
// whose entries are O(|k|^2) and whose inverse is O(|k|^-2).  Either way the
// result is Hermitian positive definite, so its rounding moves the CG's
// convergence rate, not the solution it converges to.
template <typename T, int DIM>
__device__ __forceinline__ void slot_inverse(const FK<T> &a, int e, int PB, long long in0, int lim,
                                             const Cx<double> *pin, T (&md)[DIM], Cx<T> (&mo)[3], bool &half) {
    constexpr int D = DIM;
    const int j = (int)a.d_PB.div((uint32_t)e);
    const int b = e - j * PB;
    const long long inn = in0 + b;
    #pragma unroll
    for (int c = 0; c < D; ++c) md[c] = T(0);
    mo[0] = mo[1] = mo[2] = Cx<T>{T(0), T(0)};
    half = false;
    if (!(e < PB * a.n0 && b * D < lim && !(j == 0 && inn == 0))) return;
    int m1 = 0, kh;
    if constexpr (DIM == 3) {
        m1 = (int)a.d_nh.div((uint32_t)inn);
        kh = (int)(inn - (long long)m1 * a.nh);
    } else {
        kh = (int)inn;
    }
    half = kh == 0 || (a.last_even && kh == a.nh - 1);
    Cx<double> A[3], W[3];
    A[0] = ld2(a.aa[0], j);
    W[0] = ld2(a.om[0], j);
    A[1] = pin[4 * b + 0];
    W[1] = pin[4 * b + 1];
    A[2] = DIM == 3 ? pin[4 * b + 2] : Cx<double>{0.0, 0.0};
    W[2] = DIM == 3 ? pin[4 * b + 3] : Cx<double>{1.0, 0.0};
    if constexpr (sizeof(T) == 4) {
        Cx<float> Af[3], Wf[3];
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            Af[c] = Cx<float>{float(A[c].x), float(A[c].y)};
            Wf[c] = Cx<float>{float(W[c].x), float(W[c].y)};
        }
        if (nrm(Af[0]) + nrm(Af[1]) + nrm(Af[2]) >= a.near0) {
            // dimensionless factors aa_a h_max: M~ = M h_max^2 / ch has entries
            // of order |k h_max|^2 whatever the voxel size, so the adjugate
            // neither underflows nor overflows; M^-1 = M~^-1 h_max^2 / ch
            const float hm = a.hmax_f;
            #pragma unroll
            for (int c = 0; c < 3; ++c) Af[c] = Cx<float>{Af[c].x * hm, Af[c].y * hm};
            float Md[D];
            Cx<float> Mo[3];
            core_matrix<float, DIM>(Af, Wf, 1.0f, Md, Mo);
            herm_inverse<float, D>(Md, Mo, md, mo, a.post_f);
            return;
        }
    }
    double Md[D];
    Cx<double> Mo[3];
    core_matrix<double, DIM>(A, W, a.chalf, Md, Mo);
    double Id[D];
    Cx<double> Io[3];
    herm_inverse<double, D>(Md, Mo, Id, Io);
    #pragma unroll
    for (int c = 0; c < D; ++c) md[c] = T(Id[c]);
    #pragma unroll
    for (int c = 0; c < 3; ++c) mo[c] = Cx<T>{T(Io[c].x), T(Io[c].y)};
}

// z = M^-1 r at one wavevector (md: real diagonal, mo: upper triangle of
// M^-1) and the Parseval term Re(r . conj z) in FP64.
template <typename T, int DIM>
__device__ __forceinline__ double apply_minv(const T (&md)[DIM], const Cx<T> (&mo)[3], const Cx<T> (&r)[DIM],
                                             Cx<T> (&z)[DIM]) {
    if constexpr (DIM == 3) {
        const Cx<T> o01 = mo[0], o02 = mo[1], o12 = mo[2];
        z[0] = cadd(cadd(cscale(r[0], md[0]), cmul(o01, r[1])), cmul(o02, r[2]));
        z[1] = cadd(cadd(cmulc(r[0], o01), cscale(r[1], md[1])), cmul(o12, r[2]));
        z[2] = cadd(cadd(cmulc(r[0], o02), cmulc(r[1], o12)), cscale(r[2], md[2]));
    } else {
        const Cx<T> o01 = mo[0];
        z[0] = cadd(cscale(r[0], md[0]), cmul(o01, r[1]));
        z[1] = cadd(cmulc(r[0], o01), cscale(r[1], md[1]));
    }
    double dot = 0.0;
    #pragma unroll
    for (int c = 0; c < DIM; ++c) dot += double(r[c].x) * double(z[c].x) + double(r[c].y) * double(z[c].y);
    return dot;
}

// Components of one table entry: the D real diagonal entries of M^-1, then
// the real and imaginary parts of its upper triangle (3 entries in 3D, 1 in 2D).
template <int DIM>
constexpr int kMinvComps = DIM == 3 ? 9 : 4;

// Stage the per-axis phase factors of a block's PB inner wavevector indices
// in LDS: pin[4 b + 0..3] = aa_1, om_1, aa_2, om_2 (2D: aa_1, om_1).
template <typename T, int DIM>
__device__ __forceinline__ void stage_inner_phases(const FK<T> &a, long long in0, int PB, Cx<double> *pin) {
    const long long inner = a.inner_total;
    for (int b = threadIdx.x; b < PB; b += kFftThreads) {
        const long long inn = in0 + b;
        if (inn < inner) {
            if constexpr (DIM == 3) {
                const int m1 = (int)a.d_nh.div((uint32_t)inn);
                const int kh = (int)(inn - (long long)m1 * a.nh);
                pin[4 * b + 0] = ld2(a.aa[1], m1);
                pin[4 * b + 1] = ld2(a.om[1], m1);
                pin[4 * b + 2] = ld2(a.aa[2], kh);
                pin[4 * b + 3] = ld2(a.om[2], kh);
            } else {
                pin[4 * b + 0] = ld2(a.aa[1], (int)inn);
                pin[4 * b + 1] = ld2(a.om[1], (int)inn);
            }
        }
    }
}

// The (B^*B)^-1 table of the first-axis pass: one workgroup per pencil block
// writes slot_inverse of its PB n0 wavevector slots (zeros at k = 0 and past
// the last pencil), component-major within the block so that the pass reads
// each component with consecutive threads on consecutive words.  Built once
// per workspace and block size; every load case and iteration then reads the
// inverse instead of forming it again.
template <typename T, int DIM>
__global__ __launch_bounds__(kFftThreads) void k_first_table(FK<T> a) {
    constexpr int D = DIM;
    constexpr int NC = kMinvComps<DIM>;
    const int blk = blockIdx.x;
    const int PB = a.PB;
    const long long in0 = (long long)blk * PB;
    const int lim = (int)min((long long)PB, a.inner_total - in0) * D;
    const int cntk = PB * a.n0;
    __shared__ Cx<double> pin[4 * 32];
    stage_inner_phases<T, DIM>(a, in0, PB, pin);
    __syncthreads();
    T *tb = a.minv + (long long)blk * NC * cntk;
    for (int e = threadIdx.x; e < cntk; e += kFftThreads) {
        T md[D];
        Cx<T> mo[3];
        bool half;
        slot_inverse<T, DIM>(a, e, PB, in0, lim, pin, md, mo, half);
        const int pos = minv_pos(e, a.minv_q);
        #pragma unroll
        for (int c = 0; c < D; ++c) tb[c * cntk + pos] = md[c];
        #pragma unroll
        for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c) {
            tb[(D + 2 * c) * cntk + pos] = mo[c].x;
            tb[(D + 2 * c + 1) * cntk + pos] = mo[c].y;
        }
    }
}

// First axis: forward transform, per-wavevector z^ = M(k)^-1 r^ with the
// Parseval partial of r.z (mode 0), inverse transform.  Mode 1: forward only;
// mode 2: inverse only.  PERLC = false: one workgroup per block of PB pencils
// runs through every load case, forming the inverses of its wavevectors once
// (adjugate, see slot_inverse) and keeping them in registers.
// PERLC = true: one workgroup per (load case, pencil block), load cases
// fastest in the workgroup order (the L workgroups of a block run side by
// side on one XCD); the inverses are read from the table of k_first_table
// (TAB) or formed again per load case just in time.  The power-of-two PERLC
// instantiations are held to 3 waves per SIMD (at most 168 VGPRs, no spills).
template <typename T, int PPT, int DIM, int MODE, bool GEN, bool PERLC, bool TAB>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu((PERLC && !GEN) ? 3 : 1))) void k_first(FK<T> a) {
    constexpr int NT = kFftThreads;
    constexpr int D = DIM;
    constexpr int KW = (PPT + D - 1) / D;  // wavevector slots per thread: PB n0 <= PPT NT / D
    constexpr int KC = PERLC ? 1 : KW;     // cached slots
    __shared__ Cx<T> buf[PPT * NT];
    __shared__ double red[NT / 64];
    int blk, lc0, lc1;
    if constexpr (PERLC) {
        const int t = xcd_remap(blockIdx.x, a.total);
        blk = t / a.L;
        lc0 = t - blk * a.L;
        lc1 = lc0 + 1;
        if (a.st && !a.st[lc0].active) return;
    } else {
        blk = xcd_remap(blockIdx.x, a.total);
        lc0 = 0;
        lc1 = a.L;
    }
    const int PB = a.PB;
    const int nb = PB * D;
    const int n0 = a.n0;
    const long long inner = a.inner_total;
    const long long in0 = (long long)blk * PB;
    const int lim = (int)min((long long)PB, inner - in0) * D;
    const int cnt = nb * n0;
    // dynamic LDS: twiddles of axis 0, then (mode 0) the phase factors of this
    // block's PB inner wavevector indices; the axis-0 phase factors are read
    // from the plan's tables (once per wavevector slot, L2-resident)
    Cx<T> *twl = reinterpret_cast<Cx<T> *>(feh_dyn_lds);
    const int tw_bytes = ((n0 * (int)sizeof(Cx<T>) + 15) / 16) * 16;
    Cx<double> *pin = reinterpret_cast<Cx<double> *>(reinterpret_cast<char *>(feh_dyn_lds) + tw_bytes);  // [PB][4]: aa1, om1, aa2, om2 (2D: aa1, om1)
    stage(twl, a.tw, n0);
    // per cached slot: real diagonal of M^-1, then its upper triangle (complex)
    T Mid[KC][D];
    Cx<T> Mio[KC][DIM == 3 ? 3 : 1];
    unsigned half_w = 0;  // bit kw: wavevector counted once in the half-spectrum Parseval sum
    if constexpr (MODE == 0 && !TAB) {
        stage_inner_phases<T, DIM>(a, in0, PB, pin);
        __syncthreads();
        if constexpr (!PERLC) {
            #pragma unroll
            for (int kw = 0; kw < KW; ++kw) {
                T md[D];
                Cx<T> mo[3];
                bool half;
                slot_inverse<T, DIM>(a, threadIdx.x + kw * NT, PB, in0, lim, pin, md, mo, half);
                if (half) half_w |= 1u << kw;
                #pragma unroll
                for (int c = 0; c < D; ++c) Mid[kw][c] = md[c];
                #pragma unroll
                for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c) Mio[kw][c] = mo[c];
            }
        }
    }
    for (int lc = lc0; lc < lc1; ++lc) {
        if (!PERLC && a.st && !a.st[lc].active) continue;
        // the thread index passes through an empty asm statement so that the
        // index arithmetic is redone per load case instead of being hoisted
        // out of the loop into registers
        int tx = threadIdx.x;
        asm volatile("" : "+v"(tx));
        const long long boff = ((long long)lc * n0 * inner + in0) * D;
        Cx<T> *base = a.spec + boff;
        {
            const Cx<T> *src = (a.spec_in ? a.spec_in : a.spec) + boff;
            Cx<T> v[PPT];
            #pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int e0 = tx + k * NT;
                const int e = e0 < cnt ? e0 : 0;
                const int j = (int)a.nbd.div((uint32_t)e);
                const int bc = e - j * nb;
                v[k] = src[(long long)j * inner * D + (bc < lim ? bc : lim - 1)];
            }
            #pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int e0 = tx + k * NT;
                const int j = (int)a.nbd.div((uint32_t)e0);
                const int bc = e0 - j * nb;
                if (e0 < cnt) buf[e0] = (bc < lim) ? v[k] : Cx<T>{T(0), T(0)};
            }
        }
        __syncthreads();
        if (MODE != 2) lds_fft<T, PPT, GEN>(buf, nb, a.nbd, a.ax, twl, 1, false, tx);
        double acc = 0.0;
        if constexpr (MODE == 0) {
            #pragma unroll
            for (int kw = 0; kw < KW; ++kw) {
                const int e = tx + kw * NT;
                const int j = (int)a.d_PB.div((uint32_t)e);
                const int b = e - j * PB;
                if (e < PB * n0 && b * D < lim) {
                    T md[D];
                    Cx<T> mo[3];
                    bool half;
                    if constexpr (TAB) {
                        const int cntk = PB * n0;
                        const T *tb = a.minv + (long long)blk * kMinvComps<DIM> * cntk + e;
                        #pragma unroll
                        for (int c = 0; c < D; ++c) md[c] = tb[c * cntk];
                        #pragma unroll
                        for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c)
                            mo[c] = Cx<T>{tb[(D + 2 * c) * cntk], tb[(D + 2 * c + 1) * cntk]};
                        // counted once in the half-spectrum Parseval sum: the
                        // last-axis index 0 and (even length) n/2
                        const long long inn = in0 + b;
                        const int kh = DIM == 3 ? (int)(inn - (long long)a.d_nh.div((uint32_t)inn) * a.nh) : (int)inn;
                        half = kh == 0 || (a.last_even && kh == a.nh - 1);
                    } else if constexpr (PERLC) {
                        slot_inverse<T, DIM>(a, e, PB, in0, lim, pin, md, mo, half);
                    } else {
                        #pragma unroll
                        for (int c = 0; c < D; ++c) md[c] = Mid[kw][c];
                        #pragma unroll
                        for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c) mo[c] = Mio[kw][c];
                        half = (half_w >> kw) & 1u;
                    }
                    Cx<T> *pt = buf + j * nb + b * D;
                    Cx<T> r[D], z[D];
                    #pragma unroll
                    for (int c = 0; c < D; ++c) r[c] = pt[c];
                    const double dot = apply_minv<T, DIM>(md, mo, r, z);
                    #pragma unroll
                    for (int c = 0; c < D; ++c) pt[c] = z[c];
                    acc += half ? dot : 2.0 * dot;
                }
            }
            __syncthreads();
        }
        if (MODE != 1) lds_fft<T, PPT, GEN>(buf, nb, a.nbd, a.ax, twl, 1, true, tx);
        {
            Cx<T> v[PPT];
            #pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int e0 = tx + k * NT;
                v[k] = buf[e0 < cnt ? e0 : 0];
            }
            #pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int e0 = tx + k * NT;
                const int j = (int)a.nbd.div((uint32_t)e0);
                const int bc = e0 - j * nb;
                if (e0 < cnt && bc < lim) base[(long long)j * inner * D + bc] = v[k];
            }
        }
        if (MODE == 0 && a.partial) {
            const double s = block_sum<NT>(acc, red);
            if (threadIdx.x == 0) a.partial[(long long)lc * a.part_stride + blk] = s * a.invN;
        }
        __syncthreads();  // the next load case reuses buf
    }
}

// Pencils per block of the compile-time first-axis pass (N = n0): N PB D
// points per workgroup, 24 per thread in FP32 3D.
template <typename T, int N>
constexpr int ct_first_pencils() { return (sizeof(T) == 4 ? 2048 : 1024) / N; }

// First axis with the compile-time transform, the CG's fused pass only
// (forward, z = M^-1 r with the inverse table and the Parseval partial,
// inverse): one workgroup per (pencil block, load case), load cases fastest,
// as k_first with PERLC and TAB.  LDS row m0 holds the block's PB D values of
// that row in the global order (pencil-major, the D components of a
// wavevector together): the transforms run over PB D batches of one
// sub-problem, and the staging, the M^-1 step and the store take consecutive
// LDS words across the lanes of a wavefront.
template <typename T, int N, int DIM>
__global__ __launch_bounds__(kFftThreads) void k_first_ct(FK<T> a) {
    constexpr int NT = kFftThreads, D = DIM;
    constexpr int PB = ct_first_pencils<T, N>();
    constexpr int LPB = ct_log2(PB);
    constexpr int NB = PB * D;            // values per LDS row
    constexpr int RS = NT / PB;           // rows per staging sweep
    constexpr int NC = kMinvComps<DIM>;
    constexpr int CNTK = PB * N;          // wavevector slots of the block
    static_assert(NT % PB == 0 && N % RS == 0, "staging covers whole rows");
    constexpr int NR = N / RS;            // rows per thread: g + RS i
    // The forward transform's first pass (no twiddles) has its butterfly q
    // on rows q + (N / R) c and writes rows q + (N / R) d: with R = NR these
    // are the thread's own staging rows for q = g, so the pass runs on the
    // loaded values and the staging store writes its outputs.
    constexpr bool FUSE_FIRST = ct_radix_at(N, 0) == NR;
    // The inverse transform's last pass (M = 1) has butterfly p on rows
    // R p + c and writes rows p + (N / R) d: the butterflies p = g + RS k,
    // k < KB, produce exactly the thread's rows, so the pass ends in the
    // registers the global store takes.
    constexpr int SL = ct_npass(N) - 1, RL = ct_radix_at(N, SL);
    constexpr int KB = N / (RL * RS);
    constexpr bool FUSE_LAST = SL >= 1 && KB >= 1 && KB * RL == NR && ct_lstar(N, SL) * RL == N;
    __shared__ Cx<T> buf[N * NB];
    __shared__ Cx<T> twl[N];
    __shared__ double red[NT / 64];
    const int t = xcd_remap(blockIdx.x, a.total);
    const int blk = t / a.L;
    const int lc = t - blk * a.L;
    if (a.st && !a.st[lc].active) return;
    const unsigned inner = (unsigned)a.inner_total;
    const unsigned in0 = (unsigned)blk * PB;
    const int lim = min(PB, (int)(inner - in0));
    const int limD = lim * D;             // valid values per row
    const unsigned rowD = inner * D;      // complex values between consecutive m0
    Cx<T> *base = a.spec + ((long long)lc * N * inner + in0) * D;
    const Cx<T> *src = (a.spec_in ? a.spec_in : a.spec) + ((long long)lc * N * inner + in0) * D;
    for (int i = threadIdx.x; i < N; i += NT) twl[i] = a.tw[i];
    // staging slot (i, j): row m0 = g + RS i, value r = lane + PB j of the row
    const int lane = threadIdx.x & (PB - 1), g = threadIdx.x >> LPB;
    {
        Cx<T> v[NR][D];
        #pragma unroll
        for (int i = 0; i < NR; ++i) {
            #pragma unroll
            for (int j = 0; j < D; ++j) {
                const int r = lane + PB * j;
                const int rc = r < limD ? r : limD - 1;
                v[i][j] = src[__umul24((unsigned)(g + RS * i), rowD) + (unsigned)rc];
            }
        }
        #pragma unroll
        for (int j = 0; j < D; ++j) {
            const int r = lane + PB * j;
            Cx<T> x[NR];
            #pragma unroll
            for (int i = 0; i < NR; ++i) x[i] = r < limD ? v[i][j] : Cx<T>{T(0), T(0)};
            // radices 2, 4 and 8 take no twiddles from the table
            if constexpr (FUSE_FIRST) Dft<T, NR>::run(x, false, twl, 1, N);
            #pragma unroll
            for (int i = 0; i < NR; ++i) buf[(g + RS * i) * NB + r] = x[i];
        }
    }
    __syncthreads();
    ct_passes<T, N, NB, 1, FUSE_FIRST ? 1 : 0, false, 1, NB>(buf, twl);
    double acc = 0.0;
    {
        // each table component arrives in one 16-byte load of Q slots per
        // round; the table interleaves the slots (minv_pos) so that vector
        // element qq of the lanes of a wavefront covers 64 consecutive slots
        constexpr int Q = 16 / (int)sizeof(T);
        constexpr int RUN = 64 * Q;
        static_assert(CNTK % (NT * Q) == 0, "whole rounds of slots");
        typedef T TV __attribute__((ext_vector_type(Q)));
        const T *tb0 = a.minv + (long long)blk * NC * CNTK;
        const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
        #pragma unroll
        for (int k = 0; k < CNTK / (NT * Q); ++k) {
            const int run0 = (wv + k * (NT / 64)) * RUN;
            TV tv[NC];
            #pragma unroll
            for (int c = 0; c < NC; ++c) tv[c] = *reinterpret_cast<const TV *>(tb0 + c * CNTK + run0 + l * Q);
            #pragma unroll
            for (int qq = 0; qq < Q; ++qq) {
                const int e = run0 + qq * 64 + l;
                const int m0 = e >> LPB, b = e & (PB - 1);
                if (b < lim) {
                    T md[D];
                    Cx<T> mo[3];
                    #pragma unroll
                    for (int c = 0; c < D; ++c) md[c] = tv[c][qq];
                    #pragma unroll
                    for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c) mo[c] = Cx<T>{tv[D + 2 * c][qq], tv[D + 2 * c + 1][qq]};
                    const unsigned inn = in0 + b;
                    const int kh = DIM == 3 ? (int)(inn - a.d_nh.div(inn) * (unsigned)a.nh) : (int)inn;
                    const bool half = kh == 0 || (a.last_even && kh == a.nh - 1);
                    Cx<T> *pt = buf + m0 * NB + b * D;
                    Cx<T> r[D], z[D];
                    #pragma unroll
                    for (int c = 0; c < D; ++c) r[c] = pt[c];
                    const double dot = apply_minv<T, DIM>(md, mo, r, z);
                    #pragma unroll
                    for (int c = 0; c < D; ++c) pt[c] = z[c];
                    acc += half ? dot : 2.0 * dot;
                }
            }
        }
    }
    __syncthreads();
    ct_passes<T, N, NB, 1, 0, true, 1, NB, FUSE_LAST ? SL : SL + 1>(buf, twl);
    {
        Cx<T> v[NR][D];
        #pragma unroll
        for (int j = 0; j < D; ++j) {
            const int r = lane + PB * j;
            if constexpr (FUSE_LAST) {
                #pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int pp = g + RS * k;
                    Cx<T> x[RL];
                    #pragma unroll
                    for (int cc = 0; cc < RL; ++cc) x[cc] = buf[(RL * pp + cc) * NB + r];
                    #pragma unroll
                    for (int cc = 1; cc < RL; ++cc) x[cc] = cmul(x[cc], twid(twl, 1, cc * pp, true));
                    Dft<T, RL>::run(x, true, twl, 1, N);
                    #pragma unroll
                    for (int d = 0; d < RL; ++d) v[k + KB * d][j] = x[d];
                }
            } else {
                #pragma unroll
                for (int i = 0; i < NR; ++i) v[i][j] = buf[(g + RS * i) * NB + r];
            }
        }
        #pragma unroll
        for (int i = 0; i < NR; ++i) {
            #pragma unroll
            for (int j = 0; j < D; ++j) {
                const int r = lane + PB * j;
                if (r < limD) base[__umul24((unsigned)(g + RS * i), rowD) + (unsigned)r] = v[i][j];
            }
        }
    }
    if (a.partial) {
        const double s = block_sum<NT>(acc, red);
        if (threadIdx.x == 0) a.partial[(long long)lc * a.part_stride + blk] = s * a.invN;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool pow2_len(int n) { return n > 0 && (n & (n - 1)) == 0; }

template <typename T>
FK<T> base_args(const feh_plan &p, const FftArgs &fa) {
    FK<T> a{};
    a.r = static_cast<const T *>(fa.r);
    a.q = static_cast<const T *>(fa.q);
    a.r_out = static_cast<T *>(fa.r_out);
    a.spec = static_cast<Cx<T> *>(fa.spec);
    a.spec_in = static_cast<const Cx<T> *>(fa.spec_in);
    a.z = static_cast<T *>(fa.z);
    a.p_upd = static_cast<T *>(fa.p_upd);
    a.u_upd = static_cast<T *>(fa.u_upd);
    a.partial = fa.partial;
    a.st = fa.state;
    a.dim = p.dim;
    a.D = fa.comps > 0 ? fa.comps : p.dim;
    a.L = p.L;
    a.n0 = (int)p.n[0];
    a.n1 = p.dim == 3 ? (int)p.n[1] : 1;
    a.nlast = (int)p.n[p.dim - 1];
    a.nh = (int)p.nh;
    a.N = p.N;
    a.rows = p.N / a.nlast;
    a.inner_total = p.dim == 3 ? (long long)p.n[1] * p.nh : p.nh;
    a.last_even = p.last_even ? 1 : 0;
    a.part_stride = (int)p.part_stride;
    a.out_scale = fa.out_scale;
    a.invN = 1.0 / (double)p.N;
    const double vol = p.dim == 3 ? (fa.unit_volume ? 1.0 : p.h[0] * p.h[1] * p.h[2]) / 6.0
                                  : (fa.unit_volume ? 1.0 : p.h[0] * p.h[1]) / 2.0;
    a.chalf = 0.5 * vol;
    double hmax = 0.0;
    for (int ax = 0; ax < p.dim; ++ax) hmax = std::max(hmax, p.h[ax]);
    a.near0 = (float)(0.0625 / (hmax * hmax));  // |k| h_max < 1/4
    a.hmax_f = (float)hmax;
    a.post_f = (float)(hmax * hmax / a.chalf);
    a.tw_last = p.ptr<const Cx<T>>(p.off_tw[p.dim - 1]);
    for (int ax = 0; ax < 3; ++ax) {
        a.om[ax] = p.ptr<const double>(p.off_om[ax]);
        a.aa[ax] = p.ptr<const double>(p.off_aa[ax]);
    }
    a.d_D = FastDiv::make((uint32_t)a.D);
    a.d_nh = FastDiv::make((uint32_t)a.nh);
    a.d_nhD = FastDiv::make((uint32_t)(a.nh * a.D));
    return a;
}

template <typename T>
constexpr int ppt() { return sizeof(T) == 4 ? 24 : 16; }

// LDS of a last- or middle-axis pass whose tile holds `cnt` points, in
// bytes (static tile plus dynamic part).  Power-of-two lengths keep a static
// tile of the largest size (its address and the twiddle table's are then
// compile-time constants, which the radix-2/4/8 passes are measurably faster
// with); general lengths take a dynamic tile sized to the pass and rounded
// up to 16 bytes, with the twiddle table after it, so that their long rows
// leave room for a second resident workgroup.  *lbuf receives the dynamic
// tile's entries (0 for power-of-two lengths), *dyn the dynamic bytes.
template <typename T>
size_t lds_of_pass(bool gen, int cnt, int table, int *lbuf, size_t *dyn) {
    constexpr int PPT = sizeof(T) == 4 ? 24 : 16;
    constexpr int q = 16 / (int)sizeof(Cx<T>);
    *lbuf = gen ? (cnt + q - 1) / q * q : 0;
    *dyn = ((size_t)*lbuf + table) * sizeof(Cx<T>);
    const size_t stat = (gen ? 1 : (size_t)PPT * kFftThreads) * sizeof(Cx<T>);
    return stat + *dyn;
}

}  // namespace

// The last-axis passes of a plan take the compile-time transform: FP32, an
// even last axis of 128, 256 or 512 points in the default radix order, the
// default row count, D = 2 or 3 components, 32-bit byte offsets.
bool last_ct_ok(const feh_plan &p, int D) {
    const int nlast = (int)p.n[p.dim - 1];
    return p.prec == FEH_FP32 && p.tune_ct && p.tune_rr_last == 0 && p.last_even && (D == 3 || D == 2) &&
           (nlast == 128 || nlast == 256 || nlast == 512) && ct_schedule_matches(p.fft[p.dim - 1], nlast / 2) &&
           (double)D * (double)p.N * 4.0 < 4294967296.0;
}

bool cg_residual_spectral(const feh_plan &p) { return last_ct_ok(p, p.dim); }

namespace {

template <typename T>
int last_t(const feh_plan &p, const FftArgs &fa, bool inverse) {
    constexpr int PPT = ppt<T>();
    FK<T> a = base_args<T>(p, fa);
    const int last = p.dim - 1;
    a.ax = p.fft[last];
    a.tw = p.ptr<const Cx<T>>(p.off_tw[last]);
    a.tws = p.last_even ? 2 : 1;
    const int nc = a.ax.n;
    int RR = (PPT * kFftThreads) / (nc * a.D);
    if (RR < 1) return set_error(FEH_ENOTSUP, "last axis too long for the LDS transform");
    if (RR > 64) RR = 64;
    if (p.tune_rr_last > 0 && p.tune_rr_last < RR) RR = p.tune_rr_last;
    if (RR > a.rows) RR = (int)a.rows;
    a.RR = RR;
    a.nbd = FastDiv::make((uint32_t)(a.D * RR));
    a.d_nc = FastDiv::make((uint32_t)nc);
    a.nblk = (int)((a.rows + RR - 1) / RR);
    a.total = a.nblk * p.L;
    a.use_axpy = (!inverse && fa.q != nullptr && fa.state != nullptr) ? (fa.rspec ? 2 : 1) : 0;
    if (fa.rspec && (inverse || a.use_axpy != 2 || !last_ct_ok(p, a.D)))
        return set_error(FEH_EINVAL, "the spectral residual update needs the compile-time last-axis pass");
    // compile-time transform: FP32, 3D (or 2D) with an even last axis of 128,
    // 256 or 512 points in the default radix order and the default row count
    if constexpr (sizeof(T) == 4) {
      if (last_ct_ok(p, a.D)) {
        const int rr = 24 * kFftThreads / (a.nlast / 2 * a.D);  // ct_last_rows<nlast, D>()
        a.RR = rr;
        a.nblk = (int)((a.rows + rr - 1) / rr);
        a.total = a.nblk * p.L;
        const dim3 g(a.total), b(kFftThreads);
        const bool upd = inverse && fa.p_upd != nullptr;
        if (upd && (fa.u_upd == nullptr || fa.state == nullptr))
            return set_error(FEH_EINVAL, "fused CG update needs p, u and the CG state");
#define FEH_LAST_CT(NLv, Dv)                                                                                    \
        do {                                                                                                      \
            if (inverse) {                                                                                        \
                if (upd) hipLaunchKernelGGL((k_last_inv_ct<T, NLv, Dv, true>), g, b, 0, p.stream, a);             \
                else hipLaunchKernelGGL((k_last_inv_ct<T, NLv, Dv, false>), g, b, 0, p.stream, a);                \
            } else {                                                                                              \
                if (a.use_axpy == 2) hipLaunchKernelGGL((k_last_fwd_ct<T, NLv, Dv, 2>), g, b, 0, p.stream, a);    \
                else if (a.use_axpy) hipLaunchKernelGGL((k_last_fwd_ct<T, NLv, Dv, 1>), g, b, 0, p.stream, a);    \
                else hipLaunchKernelGGL((k_last_fwd_ct<T, NLv, Dv, 0>), g, b, 0, p.stream, a);                    \
            }                                                                                                     \
        } while (0)
        if (a.D == 3) {
            if (a.nlast == 512) FEH_LAST_CT(512, 3);
            else if (a.nlast == 256) FEH_LAST_CT(256, 3);
            else FEH_LAST_CT(128, 3);
        } else {
            if (a.nlast == 512) FEH_LAST_CT(512, 2);
            else if (a.nlast == 256) FEH_LAST_CT(256, 2);
            else FEH_LAST_CT(128, 2);
        }
#undef FEH_LAST_CT
        return hip_check(hipGetLastError(), "last-axis fft launch");
      }
    }
    const dim3 g(a.total), b(kFftThreads);
    const bool gen = !pow2_len(a.ax.n);
    size_t dyn;
    if (lds_of_pass<T>(gen, a.D * RR * nc, a.nlast, &a.lbuf, &dyn) > kLdsPerWorkgroup)
        return set_error(FEH_ENOTSUP, "last axis too long for the LDS transform");
    if (inverse) {
        const bool upd = fa.p_upd != nullptr;
        if (upd && (fa.u_upd == nullptr || fa.state == nullptr))
            return set_error(FEH_EINVAL, "fused CG update needs p, u and the CG state");
        if (upd) {
            if (gen) hipLaunchKernelGGL((k_last_inv<T, PPT, true, true>), g, b, dyn, p.stream, a);
            else hipLaunchKernelGGL((k_last_inv<T, PPT, false, true>), g, b, dyn, p.stream, a);
        } else {
            if (gen) hipLaunchKernelGGL((k_last_inv<T, PPT, true, false>), g, b, dyn, p.stream, a);
            else hipLaunchKernelGGL((k_last_inv<T, PPT, false, false>), g, b, dyn, p.stream, a);
        }
    } else {
        if (a.use_axpy) {
            if (gen) hipLaunchKernelGGL((k_last_fwd<T, PPT, true, true>), g, b, dyn, p.stream, a);
            else hipLaunchKernelGGL((k_last_fwd<T, PPT, false, true>), g, b, dyn, p.stream, a);
        } else {
            if (gen) hipLaunchKernelGGL((k_last_fwd<T, PPT, true, false>), g, b, dyn, p.stream, a);
            else hipLaunchKernelGGL((k_last_fwd<T, PPT, false, false>), g, b, dyn, p.stream, a);
        }
    }
    return hip_check(hipGetLastError(), "last-axis fft launch");
}

template <typename T>
int middle_t(const feh_plan &p, const FftArgs &fa, bool inverse) {
    constexpr int PPT = ppt<T>();
    FK<T> a = base_args<T>(p, fa);
    a.ax = p.fft[1];
    a.tw = p.ptr<const Cx<T>>(p.off_tw[1]);
    a.tws = 1;
    // pencils along axis 1 are indexed by the contiguous (kh, component) pairs
    const long long inner = (long long)a.nh * a.D;
    int PB = (PPT * kFftThreads) / a.n1;
    if (PB < 1) return set_error(FEH_ENOTSUP, "middle axis too long for the LDS transform");
    if (PB > 32) PB = 32;
    if (p.tune_pb_mid > 0 && p.tune_pb_mid < PB) PB = p.tune_pb_mid;
    if (PB > inner) PB = (int)inner;
    a.PB = PB;
    a.d_PB = FastDiv::make((uint32_t)PB);
    a.inner_total = inner;
    a.nblk = (int)((inner + PB - 1) / PB);
    a.total = a.nblk * a.n0 * p.L;
    // compile-time transform: the default schedule of n1 = 64 .. 512 (a power
    // of two) and the default pencil count
    if (p.tune_ct && p.tune_pb_mid == 0 && ct_schedule_matches(a.ax, a.n1) &&
        (a.n1 == 64 || a.n1 == 128 || a.n1 == 256 || a.n1 == 512)) {
        auto go = [&](auto kern, int nb) {
            a.nblk = (int)((inner + nb - 1) / nb);
            a.total = a.nblk * a.n0 * p.L;
            hipLaunchKernelGGL(kern, dim3(a.total), dim3(kFftThreads), 0, p.stream, a);
        };
        switch (a.n1 * 2 + (inverse ? 1 : 0)) {
        case 128: go(k_middle_ct<T, 64, false>, ct_batches<T, 64>()); break;
        case 129: go(k_middle_ct<T, 64, true>, ct_batches<T, 64>()); break;
        case 256: go(k_middle_ct<T, 128, false>, ct_batches<T, 128>()); break;
        case 257: go(k_middle_ct<T, 128, true>, ct_batches<T, 128>()); break;
        case 512: go(k_middle_ct<T, 256, false>, ct_batches<T, 256>()); break;
        case 513: go(k_middle_ct<T, 256, true>, ct_batches<T, 256>()); break;
        case 1024: go(k_middle_ct<T, 512, false>, ct_batches<T, 512>()); break;
        default: go(k_middle_ct<T, 512, true>, ct_batches<T, 512>()); break;
        }
        return hip_check(hipGetLastError(), "middle-axis fft launch");
    }
    size_t dyn;
    if (lds_of_pass<T>(!pow2_len(a.ax.n), PB * a.n1, a.n1, &a.lbuf, &dyn) > kLdsPerWorkgroup)
        return set_error(FEH_ENOTSUP, "middle axis too long for the LDS transform");
    if (pow2_len(a.ax.n))
        hipLaunchKernelGGL((k_middle<T, PPT, false>), dim3(a.total), dim3(kFftThreads), dyn, p.stream, a,
                           inverse ? 1 : 0);
    else
        hipLaunchKernelGGL((k_middle<T, PPT, true>), dim3(a.total), dim3(kFftThreads), dyn, p.stream, a,
                           inverse ? 1 : 0);
    return hip_check(hipGetLastError(), "middle-axis fft launch");
}

// c2c along axis 0 of a spectrum with fa.comps components, no k-solve: the
// middle-axis kernel with one outer slice, the whole axis-0 pencil set of a
// load case and the contiguous (axis 1, kh, component) index as pencils.
template <typename T>
int first_plain_t(const feh_plan &p, const FftArgs &fa, bool inverse) {
    constexpr int PPT = ppt<T>();
    FK<T> a = base_args<T>(p, fa);
    a.ax = p.fft[0];
    a.tw = p.ptr<const Cx<T>>(p.off_tw[0]);
    a.tws = 1;
    const long long inner = a.inner_total * a.D;
    const int len = a.n0;
    int PB = (PPT * kFftThreads) / len;
    if (PB < 1) return set_error(FEH_ENOTSUP, "first axis too long for the LDS transform");
    if (PB > 32) PB = 32;
    if (PB > inner) PB = (int)inner;
    a.PB = PB;
    a.d_PB = FastDiv::make((uint32_t)PB);
    a.inner_total = inner;
    a.n1 = len;   // transform length
    a.n0 = 1;     // one outer slice per load case
    a.nblk = (int)((inner + PB - 1) / PB);
    a.total = a.nblk * p.L;
    size_t dyn;
    if (lds_of_pass<T>(!pow2_len(a.ax.n), PB * len, len, &a.lbuf, &dyn) > kLdsPerWorkgroup)
        return set_error(FEH_ENOTSUP, "first axis too long for the LDS transform");
    if (pow2_len(a.ax.n))
        hipLaunchKernelGGL((k_middle<T, PPT, false>), dim3(a.total), dim3(kFftThreads), dyn, p.stream, a,
                           inverse ? 1 : 0);
    else
        hipLaunchKernelGGL((k_middle<T, PPT, true>), dim3(a.total), dim3(kFftThreads), dyn, p.stream, a,
                           inverse ? 1 : 0);
    return hip_check(hipGetLastError(), "first-axis fft launch");
}

template <typename T, int DIM>
int first_t(const feh_plan &p, const FftArgs &fa, int mode) {
    constexpr int PPT = ppt<T>();
    FK<T> a = base_args<T>(p, fa);
    a.ax = p.fft[0];
    a.tw = p.ptr<const Cx<T>>(p.off_tw[0]);
    a.tws = 1;
    const int ctpb = mode == 0 && fa.unit_volume ? first_ct_pencils(p) : 0;
    int PB = (PPT * kFftThreads) / (a.n0 * DIM);
    if (PB < 1) return set_error(FEH_ENOTSUP, "first axis too long for the LDS transform");
    if (PB > 32) PB = 32;
    // tuned value, never below a quarter of the default: the partial-sum
    // buffer holds one slot per pencil block for that size
    if (p.tune_pb_first > 0 && p.tune_pb_first < PB) PB = std::max(p.tune_pb_first, std::max(1, PB / 4));
    if (ctpb > 0) PB = ctpb;
    if (PB > a.inner_total) PB = (int)a.inner_total;
    a.PB = PB;
    a.d_PB = FastDiv::make((uint32_t)PB);
    a.nbd = FastDiv::make((uint32_t)(PB * DIM));
    a.nblk = (int)((a.inner_total + PB - 1) / PB);
    const bool perlc = first_per_load_case(p);
    a.total = perlc ? a.nblk * p.L : a.nblk;  // one block per (load case, pencils) or per pencils
    dim3 g(a.total), b(kFftThreads);
    const bool gen = !pow2_len(a.ax.n);
    const size_t dyn = ((a.n0 * sizeof(Cx<T>) + 15) / 16) * 16 + (mode == 0 ? 4 * (size_t)PB * sizeof(Cx<double>) : 0);
    if (PPT * kFftThreads * sizeof(Cx<T>) + (kFftThreads / 64) * sizeof(double) + dyn > kLdsPerWorkgroup)
        return set_error(FEH_ENOTSUP, "first axis too long for the LDS transform");
    // the CG's fused pass (element volume relative to the voxel) reads the
    // (B^*B)^-1 table, built here on the first use for this workspace and
    // block size; the test exports (true volume) form the inverses in place
    const bool tab = mode == 0 && perlc && fa.unit_volume;
    if (tab) {
        a.minv = p.ptr<T>(p.off_minv);
        // the compile-time pass reads the table with lane-interleaved slots
        a.minv_q = ctpb > 0 ? 16 / (int)sizeof(T) : 0;
        if (p.minv_ws != p.ws || p.minv_pb != PB || p.minv_q != a.minv_q) {
            hipLaunchKernelGGL((k_first_table<T, DIM>), dim3(a.nblk), b, 0, p.stream, a);
            const int rc = hip_check(hipGetLastError(), "inverse table launch");
            if (rc != FEH_OK) return rc;
            p.minv_ws = p.ws;
            p.minv_pb = PB;
            p.minv_q = a.minv_q;
        }
    }
    if (ctpb > 0) {
        switch (a.n0) {
        case 64: hipLaunchKernelGGL((k_first_ct<T, 64, DIM>), g, b, 0, p.stream, a); break;
        case 128: hipLaunchKernelGGL((k_first_ct<T, 128, DIM>), g, b, 0, p.stream, a); break;
        case 256: hipLaunchKernelGGL((k_first_ct<T, 256, DIM>), g, b, 0, p.stream, a); break;
        default: hipLaunchKernelGGL((k_first_ct<T, 512, DIM>), g, b, 0, p.stream, a); break;
        }
        return hip_check(hipGetLastError(), "first-axis fft launch");
    }
#define FEH_FIRST(M, G)                                                                                   \
    do {                                                                                                  \
        if (perlc) hipLaunchKernelGGL((k_first<T, PPT, DIM, M, G, true, false>), g, b, dyn, p.stream, a); \
        else hipLaunchKernelGGL((k_first<T, PPT, DIM, M, G, false, false>), g, b, dyn, p.stream, a);      \
    } while (0)
    switch (mode * 2 + (gen ? 1 : 0)) {
    case 0:
        if (tab) hipLaunchKernelGGL((k_first<T, PPT, DIM, 0, false, true, true>), g, b, dyn, p.stream, a);
        else FEH_FIRST(0, false);
        break;
    case 1:
        if (tab) hipLaunchKernelGGL((k_first<T, PPT, DIM, 0, true, true, true>), g, b, dyn, p.stream, a);
        else FEH_FIRST(0, true);
        break;
    case 2: FEH_FIRST(1, false); break;
    case 3: FEH_FIRST(1, true); break;
    case 4: FEH_FIRST(2, false); break;
    default: FEH_FIRST(2, true); break;
    }
#undef FEH_FIRST
    return hip_check(hipGetLastError(), "first-axis fft launch");
}

template <typename T>
int first_dispatch(const feh_plan &p, const FftArgs &fa, int mode) {
    return p.dim == 3 ? first_t<T, 3>(p, fa, mode) : first_t<T, 2>(p, fa, mode);
}

}  // namespace

// Default first-axis layout: one workgroup per (load case, pencil block) when
// the axis length is a power of two.  That variant forms the inverses again per
// load case but fits 3 waves per SIMD (FP32; 2 in FP64, bound by LDS) against 2
// (FP32) or 1 (FP64) for the register-cached variant, and runs faster at every
// measured size.  General lengths keep the cached variant (both hold about as
// many registers there).
bool first_per_load_case(const feh_plan &p) {
    if (p.tune_first_perlc != 0) return p.tune_first_perlc > 0;
    return pow2_len((int)p.n[0]);
}

// Pencils per block of the compile-time first-axis pass of the CG, or 0 when
// the plan's shape or schedule has none: a power-of-two axis 0 of 64 to 512
// points in the default radix order, the default layout (one workgroup
// per load case) and block size, and offsets that fit the 24-bit products
// of the staging.
int first_ct_pencils(const feh_plan &p) {
    const int n0 = (int)p.n[0];
    if (!p.tune_ct || p.tune_pb_first != 0 || !first_per_load_case(p)) return 0;
    if (!(n0 == 64 || n0 == 128 || n0 == 256 || n0 == 512) || !ct_schedule_matches(p.fft[0], n0)) return 0;
    const long long inner = p.dim == 3 ? p.n[1] * p.nh : p.nh;
    const long long rowD = inner * p.dim;
    if (rowD >= (1 << 24) || rowD * n0 >= (1ll << 31)) return 0;
    return (p.prec == FEH_FP32 ? 2048 : 1024) / n0;
}

int first_pencils_default(const feh_plan &p) {
    const int PPT = p.prec == FEH_FP32 ? 24 : 16;
    int PB = (PPT * kFftThreads) / (int)(p.n[0] * p.dim);
    if (PB < 1) PB = 1;
    if (PB > 32) PB = 32;
    return PB;
}

int first_num_parts(const feh_plan &p) {
    int PB = first_pencils_default(p);
    // tuned value, never below a quarter of the default: the partial-sum
    // buffer holds one slot per pencil block for that size
    if (p.tune_pb_first > 0 && p.tune_pb_first < PB) PB = std::max(p.tune_pb_first, std::max(1, PB / 4));
    if (const int ct = first_ct_pencils(p)) PB = ct;  // the CG's fused pass
    const long long inner = p.dim == 3 ? p.n[1] * p.nh : p.nh;
    if (PB > inner) PB = (int)inner;
    return (int)((inner + PB - 1) / PB);
}

int launch_forward_last(const feh_plan &p, const FftArgs &a) {
    return p.prec == FEH_FP64 ? last_t<double>(p, a, false) : last_t<float>(p, a, false);
}
int launch_inverse_last(const feh_plan &p, const FftArgs &a) {
    return p.prec == FEH_FP64 ? last_t<double>(p, a, true) : last_t<float>(p, a, true);
}
int launch_middle(const feh_plan &p, const FftArgs &a, bool inverse) {
    return p.prec == FEH_FP64 ? middle_t<double>(p, a, inverse) : middle_t<float>(p, a, inverse);
}
int launch_first_fused(const feh_plan &p, const FftArgs &a) {
    return p.prec == FEH_FP64 ? first_dispatch<double>(p, a, 0) : first_dispatch<float>(p, a, 0);
}
int launch_first_plain(const feh_plan &p, const FftArgs &a, bool inverse) {
    return p.prec == FEH_FP64 ? first_plain_t<double>(p, a, inverse) : first_plain_t<float>(p, a, inverse);
}
int launch_first(const feh_plan &p, const FftArgs &a, bool inverse) {
    const int mode = inverse ? 2 : 1;
    return p.prec == FEH_FP64 ? first_dispatch<double>(p, a, mode) : first_dispatch<float>(p, a, mode);
}

}  // namespace feh
