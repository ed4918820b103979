// Device-side FFT building blocks for gfx950: register-resident small DFTs
// and a mixed-radix Stockham (self-sorting) pass loop that exchanges data
// between passes through LDS.
//
// A batch of transforms shares one LDS buffer.  Thread t of a transform owns
// butterfly t of every pass (threads t >= n / radix idle in that pass).  Pass p
// with radix R and Ns = product of the radices before it reads
//     x[t + r n/R],  r < R,
// multiplies input r by W_{Ns R}^{(t mod Ns) r}, runs an R-point DFT and writes
//     y[(t - t mod Ns) R + (t mod Ns) + r Ns].
// The first pass therefore reads x[t + r n/R0] (so it can be loaded straight
// from global memory into registers) and the last pass produces its outputs in
// natural order at t + r n/R_last (so it can be stored straight to global
// memory, or fed to an element-wise update and then to the first pass of
// another transform whose first radix equals R_last).
#pragma once

#include <hip/hip_runtime.h>
#include "kw_internal.h"

namespace kw {

// --- compile-time trigonometry (double, Taylor series on [-pi, pi]) ---------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int i = 1; i < 24; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 24; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
constexpr double ct_angle(long m, long n) {
    long q = m % n;
    if (q < 0) q += n;
    double a = 2.0 * kPi * (double)q / (double)n;
    if (a > kPi) a -= 2.0 * kPi;
    return a;
}
// exp(-2 pi i m / n) (forward) or its conjugate (inverse)
template <long M, long N, bool INV>
struct CTw {
    static constexpr float re = (float)ct_cos(ct_angle(M, N));
    static constexpr float im = (float)(INV ? ct_sin(ct_angle(M, N)) : -ct_sin(ct_angle(M, N)));
};

// --- complex helpers -----------------------------------------------------------
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 c_rot(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
template <long M, long N, bool INV>
__device__ __forceinline__ float2 c_mul_ct(float2 a) {
    constexpr float c = CTw<M, N, INV>::re, s = CTw<M, N, INV>::im;
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// --- register DFTs on v[O + S*i], i < R, results in natural order ------------
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
    template <int S, int O, int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        float2 a = v[O], b = v[O + S];
        v[O] = c_add(a, b);
        v[O + S] = c_sub(a, b);
    }
};

template <bool INV> struct Dft<4, INV> {
    template <int S, int O, int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        float2 t0 = c_add(v[O], v[O + 2 * S]);
        float2 t1 = c_sub(v[O], v[O + 2 * S]);
        float2 t2 = c_add(v[O + S], v[O + 3 * S]);
        float2 t3 = c_rot<INV>(c_sub(v[O + S], v[O + 3 * S]));
        v[O] = c_add(t0, t2);
        v[O + 2 * S] = c_sub(t0, t2);
        v[O + S] = c_add(t1, t3);
        v[O + 3 * S] = c_sub(t1, t3);
    }
};

template <bool INV> struct Dft<3, INV> {
    template <int S, int O, int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        // X0 = a+b+c;  X1,2 = a - (b+c)/2 -+ i (sqrt3/2)(b-c)   (forward)
        constexpr float h = 0.86602540378443864676f;
        float2 a = v[O], b = v[O + S], c = v[O + 2 * S];
        float2 s = c_add(b, c);
        float2 d = c_sub(b, c);
        float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
        float2 r = c_scale(c_rot<INV>(d), h);
        v[O] = c_add(a, s);
        v[O + S] = c_add(m, r);
        v[O + 2 * S] = c_sub(m, r);
    }
};

template <bool INV> struct Dft<5, INV> {
    template <int S, int O, int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        // Pair symmetric terms: X_k = x0 + sum_{j=1,2} (x_j + x_{5-j}) cos(2 pi jk/5)
        //                          -+ i sum (x_j - x_{5-j}) sin(2 pi jk/5)
        constexpr float c1 = 0.30901699437494742410f;   // cos(2pi/5)
        constexpr float c2 = -0.80901699437494742410f;  // cos(4pi/5)
        constexpr float s1 = 0.95105651629515357212f;   // sin(2pi/5)
        constexpr float s2 = 0.58778525229247312917f;   // sin(4pi/5)
        float2 x0 = v[O];
        float2 a1 = c_add(v[O + S], v[O + 4 * S]), b1 = c_sub(v[O + S], v[O + 4 * S]);
        float2 a2 = c_add(v[O + 2 * S], v[O + 3 * S]), b2 = c_sub(v[O + 2 * S], v[O + 3 * S]);
        float2 m1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        float2 m2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        // n1 = s1 b1 + s2 b2,  n2 = s2 b1 - s1 b2  (then multiplied by -i / +i)
        float2 n1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
        float2 n2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
        n1 = c_rot<INV>(n1);
        n2 = c_rot<INV>(n2);
        v[O] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
        v[O + S] = c_add(m1, n1);
        v[O + 4 * S] = c_sub(m1, n1);
        v[O + 2 * S] = c_add(m2, n2);
        v[O + 3 * S] = c_sub(m2, n2);
    }
};

// Composite R = A * B (Cooley-Tukey in registers):
//   1) B DFTs of length A over the stride-B subsequences,
//   2) twiddle W_R^(n2 k1),
//   3) A DFTs of length B over contiguous blocks,
//   4) transpose slot B k1 + k2 -> k1 + A k2 (register renaming).
template <int R> struct Split {
    static constexpr int A = (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : 5;
    static constexpr int B = R / A;
};

template <int A, int B, int S, int O, bool INV, int N2>
struct ComposeStage1 {
    template <int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        Dft<A, INV>::template run<S * B, O + S * N2>(v);
        ComposeStage1<A, B, S, O, INV, N2 + 1>::run(v);
    }
};
template <int A, int B, int S, int O, bool INV>
struct ComposeStage1<A, B, S, O, INV, B> {
    template <int RM> __device__ __forceinline__ static void run(float2 (&)[RM]) {}
};

template <int A, int B, int S, int O, bool INV, int K1>
struct ComposeStage3 {
    template <int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        Dft<B, INV>::template run<S, O + S * B * K1>(v);
        ComposeStage3<A, B, S, O, INV, K1 + 1>::run(v);
    }
};
template <int A, int B, int S, int O, bool INV>
struct ComposeStage3<A, B, S, O, INV, A> {
    template <int RM> __device__ __forceinline__ static void run(float2 (&)[RM]) {}
};

template <int R, int A, int B, int S, int O, bool INV, int I>
struct ComposeTwiddle {
    template <int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        constexpr int k1 = I / B, n2 = I % B;
        if constexpr (k1 > 0 && n2 > 0)
            v[O + S * (B * k1 + n2)] = c_mul_ct<(long)n2 * k1, R, INV>(v[O + S * (B * k1 + n2)]);
        ComposeTwiddle<R, A, B, S, O, INV, I + 1>::run(v);
    }
};
template <int R, int A, int B, int S, int O, bool INV>
struct ComposeTwiddle<R, A, B, S, O, INV, R> {
    template <int RM> __device__ __forceinline__ static void run(float2 (&)[RM]) {}
};

template <int R, bool INV> struct Dft {
    template <int S, int O, int RM>
    __device__ __forceinline__ static void run(float2 (&v)[RM]) {
        constexpr int A = Split<R>::A, B = Split<R>::B;
        ComposeStage1<A, B, S, O, INV, 0>::run(v);
        ComposeTwiddle<R, A, B, S, O, INV, 0>::run(v);
        ComposeStage3<A, B, S, O, INV, 0>::run(v);
        float2 tmp[R];
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) tmp[k1 + A * k2] = v[O + S * (B * k1 + k2)];
#pragma unroll
        for (int k = 0; k < R; ++k) v[O + S * k] = tmp[k];
    }
};

// Runtime radix dispatch; RM bounds the register array and the radices used.
template <bool INV, int RM>
__device__ __forceinline__ void dft_rt(int R, float2 (&v)[RM]) {
    switch (R) {
    case 2: Dft<2, INV>::template run<1, 0>(v); break;
    case 3: Dft<3, INV>::template run<1, 0>(v); break;
    case 4: Dft<4, INV>::template run<1, 0>(v); break;
    case 5: Dft<5, INV>::template run<1, 0>(v); break;
    case 6: Dft<6, INV>::template run<1, 0>(v); break;
    case 8: Dft<8, INV>::template run<1, 0>(v); break;
    case 10: Dft<10, INV>::template run<1, 0>(v); break;
    case 12: Dft<12, INV>::template run<1, 0>(v); break;
    case 15: Dft<15, INV>::template run<1, 0>(v); break;
    case 16: Dft<16, INV>::template run<1, 0>(v); break;
    default:
        if constexpr (RM >= 32) {
            switch (R) {
            case 20: Dft<20, INV>::template run<1, 0>(v); break;
            case 24: Dft<24, INV>::template run<1, 0>(v); break;
            case 25: Dft<25, INV>::template run<1, 0>(v); break;
            case 30: Dft<30, INV>::template run<1, 0>(v); break;
            case 32: Dft<32, INV>::template run<1, 0>(v); break;
            default: break;
            }
        }
        break;
    }
}

// --- LDS addressing ------------------------------------------------------------
// Orders the LDS accesses of one wavefront.  Its lanes run in lockstep and the
// LDS serves one wavefront's requests in order, so a transform whose threads
// all lie in one wavefront needs no s_barrier between its passes: only the
// compiler must keep the accesses on their side of this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column batches (y and z passes): element n of transform b at sh[n * tb + b];
// consecutive lanes hold consecutive b, so every access is bank-conflict free
// once tb >= 16.  A column's threads span wavefronts: block barriers.
// ld2/st2(n0, d): element n0 + d with d uniform over the block, so that only
// n0 * tb is a per-lane product (24-bit, full rate) and d * tb is scalar.
struct ColLds {
    float2 *sh;
    int tb, b;
    __device__ __forceinline__ float2 ld(int n) const { return sh[__umul24(n, tb) + b]; }
    __device__ __forceinline__ void st(int n, float2 x) const { sh[__umul24(n, tb) + b] = x; }
    __device__ __forceinline__ float2 ld2(int n0, int d) const { return sh[__umul24(n0, tb) + b + d * tb]; }
    __device__ __forceinline__ void st2(int n0, int d, float2 x) const {
        sh[__umul24(n0, tb) + b + d * tb] = x;
    }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};
// Row batches (x passes): transform b occupies a padded row; one pad slot per
// 16 elements spreads the strided Stockham writes over the banks.  `wave`:
// the L threads of a row are lanes of one wavefront (L divides the wavefront
// size and rows start at multiples of L), so the passes synchronise only the
// wavefront; the flag is uniform over the block.
struct RowLds {
    float2 *sh;
    int base;
    bool wave;
    __device__ __forceinline__ float2 ld(int n) const { return sh[base + n + (n >> 4)]; }
    __device__ __forceinline__ void st(int n, float2 x) const { sh[base + n + (n >> 4)] = x; }
    __device__ __forceinline__ float2 ld2(int n0, int d) const { return ld(n0 + d); }
    __device__ __forceinline__ void st2(int n0, int d, float2 x) const { st(n0 + d, x); }
    __device__ __forceinline__ void sync() const {
        if (wave) wave_sync();
        else __syncthreads();
    }
};
// Whether the rows of L threads of a block lie within wavefronts
__device__ __forceinline__ bool rows_in_waves(int L) { return (warpSize % L) == 0; }

// --- the pass loop -----------------------------------------------------------
// On entry v[r] (r < radix[0]) holds x[t + r n/radix[0]] for t < n/radix[0].
// On exit v[r] (r < radix[np-1]) holds X[t + r n/radix[np-1]] for t < n/radix[np-1].
// Every thread of the block must call this (it contains barriers, of the block
// or of the wavefront, see RowLds); the trailing one makes the LDS buffer free
// for reuse by the same threads on return.
template <bool INV, int RM, class Lds>
__device__ __forceinline__ void fft_run(const FftPlan &P, const float2 *__restrict__ tw, int t,
                                        const Lds &lds, float2 (&v)[RM]) {
    int Ns = 1;
    for (int p = 0; p < P.np; ++p) {
        const int R = plan_radix(P, p);
        const int nb = P.n / R;
        const bool act = t < nb;
        if (p > 0) {
            lds.sync();
            if (act) {
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r < R) v[r] = lds.ld2(t, r * nb);
            }
            lds.sync();
        }
        if (act) {
            const int k = t % Ns;
            if (Ns > 1) {
                const int kst = __umul24(k, P.n / (Ns * R));
#pragma unroll
                for (int r = 1; r < RM; ++r) {
                    if (r < R) {
                        const float2 w = tw[kst * r];
                        v[r] = INV ? c_mulc(v[r], w) : c_mul(v[r], w);
                    }
                }
            }
            dft_rt<INV, RM>(R, v);
            if (p < P.np - 1) {
                const int base = (t - k) * R + k;
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r < R) lds.st2(base, r * Ns, v[r]);
            }
        }
        Ns *= R;
    }
    lds.sync();
}


// --- fixed-width engine ---------------------------------------------------------
// Every thread owns E elements: x[t + m L], m < E, with L = n / E threads per
// transform, in the first pass and after the last pass whatever the radix
// schedule (every radix divides E).  A pass of radix R runs E/R butterflies per
// thread, j = t + b L (b < E/R); butterfly j reads x[j + r n/R], which is
// element t + L (b + r E/R) -- register b + r E/R.
// E = 4, 8, 16 serve power-of-two lengths (radices 2 to 16) and E = 32 the
// powers of 32 (radix-32 passes only); E = 12 and
// E = 20 serve lengths with a factor 3 or 5 (radices 2, 3, 4, 6, 12 and
// 2, 4, 5, 10, 20), where the butterfly's position k = j mod Ns within its
// group is no longer a bit mask.
template <int E, int R, bool INV, int Bi>
struct FixedBfly {
    template <class Lds>
    __device__ __forceinline__ static void run(float2 (&v)[E], int t, int L, int Ns, int st,
                                               const float2 *__restrict__ tw, const Lds &lds,
                                               bool write) {
        constexpr int B = E / R;
        if constexpr (Bi < B) {
            const int j = t + Bi * L;
            const int k = ((E & (E - 1)) == 0) ? (j & (Ns - 1)) : (int)((unsigned)j % (unsigned)Ns);
            if (Ns > 1) {
                const int kst = __umul24(k, st);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float2 w = tw[kst * r];
                    v[Bi + r * B] = INV ? c_mulc(v[Bi + r * B], w) : c_mul(v[Bi + r * B], w);
                }
            }
            Dft<R, INV>::template run<B, Bi>(v);
            if (write) {
                const int base = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) lds.st2(base, r * Ns, v[Bi + r * B]);
            }
            FixedBfly<E, R, INV, Bi + 1>::run(v, t, L, Ns, st, tw, lds, write);
        }
    }
};

template <int E, int R, bool INV, class Lds>
__device__ __forceinline__ void pass_fixed(float2 (&v)[E], int t, int L, int Ns, int st,
                                           const float2 *__restrict__ tw, const Lds &lds,
                                           bool write) {
    FixedBfly<E, R, INV, 0>::run(v, t, L, Ns, st, tw, lds, write);
}

// A set of radices: bit q stands for radix q (0: every radix that divides E)
using RadixSet = unsigned long long;
constexpr RadixSet radix_bit(int q) { return 1ull << q; }

// One pass of radix R, where R is known to be in the set RS: only the passes
// of RS are compiled (the largest radix first)
template <int E, RadixSet RS, bool INV, class Lds>
__device__ __forceinline__ void pass_in_set(int R, float2 (&v)[E], int t, int L, int Ns, int st,
                                            const float2 *__restrict__ tw, const Lds &lds,
                                            bool write) {
    constexpr int q = 63 - __builtin_clzll(RS);
    if constexpr ((RS & (RS - 1)) == 0) {
        pass_fixed<E, q, INV>(v, t, L, Ns, st, tw, lds, write);
    } else {
        if (R == q) pass_fixed<E, q, INV>(v, t, L, Ns, st, tw, lds, write);
        else pass_in_set<E, RS & ~radix_bit(q), INV>(R, v, t, L, Ns, st, tw, lds, write);
    }
}

// On entry v[m] = x[t + m L]; on exit v[m] = X[t + m L] (m < E, t < L).
// RS: the radices of the plans this instantiation runs (0: any that divide E)
template <bool INV, int E, RadixSet RS, class Lds>
__device__ __forceinline__ void fft_fixed(const FftPlan &P, const float2 *__restrict__ tw, int t,
                                          const Lds &lds, float2 (&v)[E]) {
    const int L = P.L;
    int Ns = 1;
    for (int p = 0; p < P.np; ++p) {
        const int R = plan_radix(P, p);
        if (p > 0) {
            lds.sync();
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds.ld2(t, m * L);
            lds.sync();
        }
        const int st = P.n / (Ns * R);
        const bool write = p < P.np - 1;
        // (a plan holds only radices that divide E)
        if constexpr (RS != 0 || E == 32) {
            // Instantiations for a set of radices, and the 32-wide engine,
            // which runs radix-32 passes only: the code of the radices a plan
            // does not use (a switch on the pass's radix) raises the register
            // count of every kernel built on the engine, though it never runs.
            // Measured without it: the 32-wide y pass 206 -> 124 registers and
            // its merged absorption z pass 284 -> 60 bytes a thread spilled;
            // the 16-wide y pass 106 -> 68, the 8-wide velocity x pass
            // 114 -> 96, the 12-wide three-group density pass 98 -> 89.
            pass_in_set<E, (RS != 0 ? RS : radix_bit(32)), INV>(R, v, t, L, Ns, st, tw, lds, write);
        } else
        switch (R) {
        case 2: pass_fixed<E, 2, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 4: if constexpr (E % 4 == 0) pass_fixed<E, 4, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 8: if constexpr (E % 8 == 0) pass_fixed<E, 8, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 16: if constexpr (E % 16 == 0) pass_fixed<E, 16, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 32: if constexpr (E % 32 == 0) pass_fixed<E, 32, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 3: if constexpr (E % 3 == 0) pass_fixed<E, 3, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 6: if constexpr (E % 6 == 0) pass_fixed<E, 6, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 12: if constexpr (E % 12 == 0) pass_fixed<E, 12, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 5: if constexpr (E % 5 == 0) pass_fixed<E, 5, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 10: if constexpr (E % 10 == 0) pass_fixed<E, 10, INV>(v, t, L, Ns, st, tw, lds, write); break;
        case 20: if constexpr (E % 20 == 0) pass_fixed<E, 20, INV>(v, t, L, Ns, st, tw, lds, write); break;
        default: break;
        }
        Ns *= R;
    }
    lds.sync();
}

// Engine policies used by the kernels.  `in_*` is the register layout of the
// input of the plan being run and `out_*` the layout of its output.  For the
// generic engine the inverse of an axis runs the reversed plan, so the output
// layout of a forward transform is the input layout of the inverse one and
// vice versa; for the fixed engine both layouts are t + m L for every plan.
template <int RM>
struct EngGeneric {
    static constexpr int E = RM;
    static constexpr bool fixed = false;
    __device__ static __forceinline__ int in_count(const FftPlan &P, int t) {
        const int R = plan_radix(P, 0);
        return t < P.n / R ? R : 0;
    }
    __device__ static __forceinline__ int in_index(const FftPlan &P, int t, int m) {
        return t + m * (P.n / plan_radix(P, 0));
    }
    __device__ static __forceinline__ int out_count(const FftPlan &P, int t) {
        const int R = plan_radix(P, P.np - 1);
        return t < P.n / R ? R : 0;
    }
    __device__ static __forceinline__ int out_index(const FftPlan &P, int t, int m) {
        return t + m * (P.n / plan_radix(P, P.np - 1));
    }
    // index distance between consecutive m of the input / output layout
    __device__ static __forceinline__ int in_step(const FftPlan &P) { return P.n / plan_radix(P, 0); }
    __device__ static __forceinline__ int out_step(const FftPlan &P) {
        return P.n / plan_radix(P, P.np - 1);
    }
    template <bool INV, class Lds>
    __device__ static __forceinline__ void run(const FftPlan &P, const float2 *tw, int t,
                                               const Lds &lds, float2 (&v)[RM]) {
        fft_run<INV, RM>(P, tw, t, lds, v);
    }
};

// RS: the radices of the plans run on this instantiation (0: any that
// divide EE)
template <int EE, RadixSet RS = 0>
struct EngFixed {
    static constexpr int E = EE;
    static constexpr bool fixed = true;
    __device__ static __forceinline__ int in_count(const FftPlan &, int) { return EE; }
    __device__ static __forceinline__ int in_index(const FftPlan &P, int t, int m) {
        return t + m * P.L;
    }
    __device__ static __forceinline__ int out_count(const FftPlan &, int) { return EE; }
    __device__ static __forceinline__ int out_index(const FftPlan &P, int t, int m) {
        return t + m * P.L;
    }
    __device__ static __forceinline__ int in_step(const FftPlan &P) { return P.L; }
    __device__ static __forceinline__ int out_step(const FftPlan &P) { return P.L; }
    template <bool INV, class Lds>
    __device__ static __forceinline__ void run(const FftPlan &P, const float2 *tw, int t,
                                               const Lds &lds, float2 (&v)[EE]) {
        fft_fixed<INV, EE, RS>(P, tw, t, lds, v);
    }
};
// plans of radix-8 (radix-16) passes only; plans of radices 8 and 4 at width
// 8; plans of radices 6 and 4 at width 12
using EngFixed8P = EngFixed<8, radix_bit(8)>;
using EngFixed16P = EngFixed<16, radix_bit(16)>;
using EngFixed8_84 = EngFixed<8, radix_bit(8) | radix_bit(4)>;
using EngFixed12_64 = EngFixed<12, radix_bit(6) | radix_bit(4)>;

}  // namespace kw
