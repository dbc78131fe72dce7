// Compile-time LDS Stockham FFT of up to NL lines of length N (radices 16, 8, 4, 2, 3).
//
// Every stage a thread loads the R inputs of up to MB butterflies, applies the
// twiddles exp(-+2 pi i r k / (Ns R)) (stage-major table tw, see
// fft_stage_index), runs the radix-R DFT in registers, and after a barrier
// stores the outputs in autosort (Stockham) order; all index arithmetic is by
// compile-time constants.  The power-of-two part uses as few stages as
// possible (radix 16 where that saves a stage over radix 8), since every stage
// costs an LDS round trip and a twiddle multiplication per point.
//
// Two LDS layouts.  The LDS serves the 32 lanes of a half wave per pass, and an
// access of 8 or 16 bytes per lane is conflict free when the element indices
// of those lanes are distinct modulo 32 (8-byte elements) or cover each
// residue modulo 16 at most twice (16-byte elements).
//  * padded (ILV = false): line l at buf[l * fft_ls(N) + fft_pad(e)], one
//    padding element after every 16, butterflies numbered line by line.  Used
//    where a workgroup holds few lines.
//  * interleaved (ILV = true): line l at buf[l * (N | 1) + e], and the lanes of
//    a half wave take the same butterfly of 32 consecutive lines, so every
//    load and store of a stage touches 32 different lines at one offset: with
//    the odd line stride these are 32 different banks.  Lines beyond the last
//    complete group of 32 are numbered line by line.
#pragma once

#include "common.h"

namespace xfft {

__host__ __device__ constexpr int fft_pad(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int fft_ls(int n) { return ((n + (n >> 4)) | 1); }   // odd line stride

// line stride and element position of the two layouts
template <bool ILV> __host__ __device__ constexpr int lds_ls(int n) { return ILV ? (n | 1) : fft_ls(n); }
template <bool ILV> __host__ __device__ constexpr int lds_pos(int e) { return ILV ? e : fft_pad(e); }

__host__ __device__ constexpr int fft_radix(int n, int stage) {
    int a = 0, m = n;
    while (m % 2 == 0) { m /= 2; ++a; }
    const bool use16 = (a + 3) / 4 < (a + 2) / 3;
    int r[16] = {};
    int ns = 0;
    if (use16) {
        for (int i = 0; i < a / 4; ++i) r[ns++] = 16;
        if (a % 4 == 3) r[ns++] = 8;
        if (a % 4 == 2) r[ns++] = 4;
        if (a % 4 == 1) r[ns++] = 2;
    } else {
        for (int i = 0; i < a / 3; ++i) r[ns++] = 8;
        if (a % 3 == 2) r[ns++] = 4;
        if (a % 3 == 1) r[ns++] = 2;
    }
    while (m % 3 == 0) { m /= 3; r[ns++] = 3; }
    return stage < ns ? r[stage] : 0;
}

// Stage-major twiddle table of the compile-time plan of length n: the R - 1
// twiddles exp(-2 pi i r k / (Ns R)), r = 1 .. R-1, of butterfly column k of
// the stage with span Ns are contiguous at Ns - 1 + k (R - 1) + r - 1, so a
// butterfly addresses them with one base and constant offsets.  Entry e
// (0 <= e < n - 1) equals exp(-2 pi i t / n) with the t returned here (-1 when
// n has no compile-time plan).
__host__ __device__ constexpr int fft_stage_index(int n, int e) {
    int ns = 1;
    for (int st = 0;; ++st) {
        const int R = fft_radix(n, st);
        if (R == 0) return -1;
        if (e < ns * R - 1) {
            const int off = e - (ns - 1), k = off / (R - 1), r = off % (R - 1) + 1;
            return r * k * (n / (ns * R));
        }
        ns *= R;
        if (ns >= n) return -1;
    }
}

// x * exp(-+2 pi i M / 16), exact for multiples of a quarter turn
template <typename T, bool INV, int M>
__device__ __forceinline__ cpx<T> rot16(cpx<T> x) {
    constexpr int m = ((M % 16) + 16) % 16;
    if constexpr (m == 0) return x;
    else if constexpr (m == 8) return {-x.x, -x.y};
    else if constexpr (m == 4) return INV ? cpx<T>{-x.y, x.x} : cpx<T>{x.y, -x.x};
    else if constexpr (m == 12) return INV ? cpx<T>{x.y, -x.x} : cpx<T>{-x.y, x.x};
    else {
        constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
        constexpr double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
        constexpr double sn[16] = {0, s1, h, c1, 1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1};
        const T c = (T)cs[m], s = (T)sn[m];
        return INV ? cpx<T>{x.x * c - x.y * s, x.y * c + x.x * s} : cpx<T>{x.x * c + x.y * s, x.y * c - x.x * s};
    }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2, cpx<T> &x3) {
    const cpx<T> t0 = cadd(x0, x2), t1 = csub(x0, x2);
    const cpx<T> t2 = cadd(x1, x3), t3 = csub(x1, x3);
    const cpx<T> t3r = INV ? cpx<T>{-t3.y, t3.x} : cpx<T>{t3.y, -t3.x};   // -+ i t3
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3r);
    x3 = csub(t1, t3r);
}

template <typename T, bool INV, int R>
__device__ __forceinline__ void dft_small(cpx<T> (&v)[16]) {
    if constexpr (R == 2) {
        const cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        dft4<T, INV>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 16) {
        // 16 = 4 x 4: length-4 DFTs over n1 (n = n2 + 4 n1), twiddles w^(n2 k1),
        // length-4 DFTs over n2; output k = k1 + 4 k2
        cpx<T> y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            y[n2][0] = v[n2]; y[n2][1] = v[n2 + 4]; y[n2][2] = v[n2 + 8]; y[n2][3] = v[n2 + 12];
            dft4<T, INV>(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
        }
        y[1][1] = rot16<T, INV, 1>(y[1][1]);
        y[1][2] = rot16<T, INV, 2>(y[1][2]);
        y[1][3] = rot16<T, INV, 3>(y[1][3]);
        y[2][1] = rot16<T, INV, 2>(y[2][1]);
        y[2][2] = rot16<T, INV, 4>(y[2][2]);
        y[2][3] = rot16<T, INV, 6>(y[2][3]);
        y[3][1] = rot16<T, INV, 3>(y[3][1]);
        y[3][2] = rot16<T, INV, 6>(y[3][2]);
        y[3][3] = rot16<T, INV, 9>(y[3][3]);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            dft4<T, INV>(y[0][k1], y[1][k1], y[2][k1], y[3][k1]);
            v[k1] = y[0][k1]; v[k1 + 4] = y[1][k1]; v[k1 + 8] = y[2][k1]; v[k1 + 12] = y[3][k1];
        }
    } else if constexpr (R == 8) {
        // even / odd halves, then X[k] = E[k] + W^k O[k], X[k+4] = E[k] - W^k O[k]
        cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<T, INV>(e0, e1, e2, e3);
        dft4<T, INV>(o0, o1, o2, o3);
        const T h = (T)0.70710678118654752440;
        // W = exp(-+ i pi / 4)
        const cpx<T> w1o = INV ? cpx<T>{h * (o1.x - o1.y), h * (o1.x + o1.y)}
                               : cpx<T>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
        const cpx<T> w2o = INV ? cpx<T>{-o2.y, o2.x} : cpx<T>{o2.y, -o2.x};
        const cpx<T> w3o = INV ? cpx<T>{-h * (o3.x + o3.y), h * (o3.x - o3.y)}
                               : cpx<T>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, w1o);
        v[5] = csub(e1, w1o);
        v[2] = cadd(e2, w2o);
        v[6] = csub(e2, w2o);
        v[3] = cadd(e3, w3o);
        v[7] = csub(e3, w3o);
    } else {
        const T c = (T)0.86602540378443864676;
        const cpx<T> a = v[0];
        const cpx<T> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        const cpx<T> m = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
        const cpx<T> it2 = INV ? cpx<T>{-c * t2.y, c * t2.x} : cpx<T>{c * t2.y, -c * t2.x};
        v[0] = cadd(a, t1);
        v[1] = cadd(m, it2);
        v[2] = csub(m, it2);
    }
}

// For power-of-two NB and NS the padded position of element e + r * M (M = NB
// for loads, NS for stores, e the butterfly's first element) is
// fft_pad(e) + r * M + (r * M) / 16 for every r < R, so each butterfly computes
// one LDS address and the R accesses use constant offsets.
template <int M> __host__ __device__ constexpr int pad_step(int r) { return r * M + ((r * M) >> 4); }

template <typename T, int N, int NL, int NT, bool INV, bool ILV = false, int STAGE = 0, int NS = 1>
__device__ __forceinline__ void fft_lines(cpx<T> *buf, const cpx<T> *__restrict__ tw, int nl = NL,
                                          int tid = threadIdx.x) {
    constexpr int R = fft_radix(N, STAGE);
    if constexpr (R != 0) {
        constexpr int LS = lds_ls<ILV>(N);
        constexpr int NB = N / R;
        constexpr int TOTAL = NL * NB;
        constexpr int MB = (TOTAL + NT - 1) / NT;
        // constant load and store offsets: always in the interleaved layout,
        // for power-of-two NB and NS in the padded one
        constexpr bool P2 = ILV || ((NB & (NB - 1)) == 0 && (NS & (NS - 1)) == 0);
        const int total = nl * NB;          // lines nl .. NL-1 are skipped
        const int full = ILV ? (nl & ~31) * NB : 0;   // butterflies of complete 32-line groups
        cpx<T> v[MB][16];
        int st[MB];                         // LDS position of each butterfly's first output
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = tid + i * NT;
            st[i] = 0;
            if ((TOTAL % NT == 0 && nl == NL) || b < total) {
                int line, jj;
                if (ILV && b < full) {
                    const int g = b >> 5;
                    jj = g % NB;
                    line = (g / NB) * 32 + (b & 31);
                } else {
                    const int bb = b - full;
                    line = full / NB + bb / NB;
                    jj = bb % NB;
                }
                const int k = jj % NS;
                const int base = (jj / NS) * NS * R + k;
                const int ld = line * LS + lds_pos<ILV>(jj);
                st[i] = line * LS + lds_pos<ILV>(base);
                const cpx<T> *twk = tw + (NS - 1) + k * (R - 1) - 1;   // twk[r], r >= 1
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cpx<T> x = ILV ? buf[ld + r * NB]
                             : P2  ? buf[ld + pad_step<NB>(r)]
                                   : buf[line * LS + fft_pad(jj + r * NB)];
                    if (NS > 1 && r > 0) {
                        cpx<T> w = twk[r];
                        if (INV) w.y = -w.y;
                        x = cmul(x, w);
                    }
                    v[i][r] = x;
                }
                dft_small<T, INV, R>(v[i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = tid + i * NT;
            if ((TOTAL % NT == 0 && nl == NL) || b < total) {
                if constexpr (ILV) {
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[st[i] + r * NS] = v[i][r];
                } else if constexpr (P2) {
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[st[i] + pad_step<NS>(r)] = v[i][r];
                } else {
                    const int line = b / NB, jj = b - line * NB;
                    const int base = (jj / NS) * NS * R + jj % NS;
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[line * LS + fft_pad(base + r * NS)] = v[i][r];
                }
            }
        }
        __syncthreads();
        fft_lines<T, N, NL, NT, INV, ILV, STAGE + 1, NS * R>(buf, tw, nl, tid);
    }
}

}  // namespace xfft
