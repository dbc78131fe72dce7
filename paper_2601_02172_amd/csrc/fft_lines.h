// Compile-time LDS Stockham FFT of NL lines of length N (radices 4, 2, 3).
//
// Line l occupies buf[l * LS + (0 .. N-1)] with LS = N + 1 (odd stride: no LDS
// bank conflicts between lines).  Every stage a thread loads the R inputs of up
// to MB butterflies, applies the twiddles exp(-+2 pi i r k / (Ns R)) (table tw of
// exp(-2 pi i t / N)), runs the radix-R DFT in registers, and after a barrier
// stores the outputs in autosort (Stockham) order; all index arithmetic is by
// compile-time constants.
#pragma once

#include "common.h"

namespace xfft {

__host__ __device__ constexpr int fft_radix(int n, int stage) {
    int m = n, s = 0;
    while (m % 4 == 0) { if (s == stage) return 4; m /= 4; ++s; }
    while (m % 2 == 0) { if (s == stage) return 2; m /= 2; ++s; }
    while (m % 3 == 0) { if (s == stage) return 3; m /= 3; ++s; }
    return 0;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft_small(cpx<T> (&v)[4], int R) {
    if (R == 2) {
        const cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        const cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const cpx<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        const cpx<T> t3r = INV ? cpx<T>{-t3.y, t3.x} : cpx<T>{t3.y, -t3.x};
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3r);
        v[3] = csub(t1, t3r);
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

template <typename T, int N, int NL, int NT, bool INV, int STAGE = 0, int NS = 1>
__device__ __forceinline__ void fft_lines(cpx<T> *buf, const cpx<T> *__restrict__ tw) {
    constexpr int R = fft_radix(N, STAGE);
    if constexpr (R != 0) {
        constexpr int LS = N + 1;
        constexpr int NB = N / R;
        constexpr int TOTAL = NL * NB;
        constexpr int MB = (TOTAL + NT - 1) / NT;
        constexpr int TWS = N / (NS * R);
        cpx<T> v[MB][4];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = threadIdx.x + i * NT;
            if (TOTAL % NT == 0 || b < TOTAL) {
                const int line = b / NB, jj = b - line * NB;
                const int k = jj % NS;
                const cpx<T> *Lp = buf + line * LS;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    cpx<T> x = Lp[jj + r * NB];
                    if (NS > 1 && r > 0) {
                        cpx<T> w = tw[r * k * TWS];
                        if (INV) w.y = -w.y;
                        x = cmul(x, w);
                    }
                    v[i][r] = x;
                }
                dft_small<T, INV>(v[i], R);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const int b = threadIdx.x + i * NT;
            if (TOTAL % NT == 0 || b < TOTAL) {
                const int line = b / NB, jj = b - line * NB;
                const int k = jj % NS;
                cpx<T> *Lp = buf + line * LS;
                const int base = (jj / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) Lp[base + r * NS] = v[i][r];
            }
        }
        __syncthreads();
        fft_lines<T, N, NL, NT, INV, STAGE + 1, NS * R>(buf, tw);
    }
}

}  // namespace xfft
