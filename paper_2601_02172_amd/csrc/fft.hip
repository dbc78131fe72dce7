// Green operator of the reference FE stiffness (eqs. constantCoefficientPreconditioner,
// GreenHermitian) applied by real 3-D FFT, in five passes over HBM:
//   x forward  r2c along x of row pairs (two real rows packed as one complex
//              line), fused with the residual update f -= alpha z;
//   y forward  complex FFT along y;
//   z + Green  complex FFT along z, per-frequency 3x3 solve with the symbol of
//              A11^0, Parseval partial of f^T G f, inverse FFT along z;
//   y inverse;
//   x inverse  c2r of row pairs fused with the CG update of d and u.
// Every line FFT is an LDS Stockham autosort transform with radices 4, 2, 3.
//
// Symbol (derived from eq. GreenHermitian for the six Kuhn elements of the
// reference voxel, identity material; real and symmetric): with
// theta_a = 2 pi xi_a / n_a, s_a = sin(theta_a / 2),
//   S_aa = 2 sum_b s_b^2 + 2 s_a^2,
//   S_ab = (2/3) s_a s_b [2 cos(phi_ab) + cos(phi_ab + theta_c)],
//   phi_ab = (theta_a + theta_b) / 2, {a, b, c} = {0, 1, 2};
// S(0) = 0 maps the zero frequency to zero (mean-free FE field).
#include "kernels.h"
#include "enriched.h"
#include "fft_lines.h"

#include <algorithm>

namespace xfft {

FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    int m = n, k = 0;
    while (m % 4 == 0) { p.radix[k++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[k++] = 2; m /= 2; }
    while (m % 3 == 0) { p.radix[k++] = 3; m /= 3; }
    p.nstages = (m == 1) ? k : -1;
    return p;
}

namespace {

constexpr int MAXB = 4;

template <typename T, bool INV>
__device__ __forceinline__ void butterfly(cpx<T> (&v)[4], int R) {
    if (R == 2) {
        const cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        const cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        const cpx<T> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
        // forward: multiply t3 by -i; inverse: by +i
        const cpx<T> t3r = INV ? cpx<T>{-t3.y, t3.x} : cpx<T>{t3.y, -t3.x};
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3r);
        v[3] = csub(t1, t3r);
    } else {  // R == 3
        const T c = (T)0.86602540378443864676;   // sqrt(3)/2
        const cpx<T> a = v[0];
        const cpx<T> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        const cpx<T> m = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
        // forward: y1 = m - i c t2, y2 = m + i c t2 (inverse swaps)
        const cpx<T> it2 = INV ? cpx<T>{-c * t2.y, c * t2.x} : cpx<T>{c * t2.y, -c * t2.x};
        v[0] = cadd(a, t1);
        v[1] = cadd(m, it2);
        v[2] = csub(m, it2);
    }
}

// In-place Stockham FFT of `nlines` lines stored at buf + line * lstride.
template <typename T, bool INV>
__device__ void lds_fft(cpx<T> *buf, int nlines, int lstride, const FftPlan &pl, const cpx<T> *__restrict__ tw) {
    const int n = pl.n;
    int Ns = 1;
    for (int st = 0; st < pl.nstages; ++st) {
        const int R = pl.radix[st];
        const int nb = n / R;
        const int total = nlines * nb;
        const int tws = n / (Ns * R);
        cpx<T> v[MAXB][4];
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int b = threadIdx.x + i * blockDim.x;
            if (b < total) {
                const int line = b / nb, jj = b - line * nb;
                const int k = jj % Ns;
                const cpx<T> *Lp = buf + line * lstride;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r < R) {
                        cpx<T> x = Lp[jj + r * nb];
                        if (r > 0) {
                            cpx<T> w = tw[r * k * tws];
                            if (INV) w.y = -w.y;
                            x = cmul(x, w);
                        }
                        v[i][r] = x;
                    }
                }
                butterfly<T, INV>(v[i], R);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int b = threadIdx.x + i * blockDim.x;
            if (b < total) {
                const int line = b / nb, jj = b - line * nb;
                const int k = jj % Ns;
                cpx<T> *Lp = buf + line * lstride;
                const int base = (jj / Ns) * Ns * R + k;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r < R) Lp[base + r * Ns] = v[i][r];
            }
        }
        __syncthreads();
        Ns *= R;
    }
}

struct FftArgs {
    int n0, n1, n2, nh;
    int nhs;                 // row stride of the spectrum (>= nh; padded in the [c][kz][ky][kx] layout)
    int64_t N, specN;        // nodes; complex entries per component spectrum... per rhs: 3 * specN
    const Flags *flags;
    int parity;
    const Scalars *scal;
    double *partial;
    int nslots, slot0;
};

__device__ __forceinline__ bool active_rhs(const FftArgs &A, int r) {
    return A.flags == nullptr || A.flags[r].active[A.parity] != 0;
}

// ---------------------------------------------------------------- x forward (r2c)
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_fwd(FftArgs A, FftPlan pl, const cpx<T> *tw, T *f, const T *z,
                                                    cpx<T> *spec, int pairs_per_block) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int r = blockIdx.y;
    if (!active_rhs(A, r)) return;
    const int n0 = A.n0, nh = A.nh, nhs = A.nhs;
    const int lstride = n0 + 1;
    const int64_t npairs = (int64_t)3 * A.n2 * A.n1 / 2;
    const T alpha = z ? (T)A.scal[r].alpha : (T)0;
    T *fr = f + (int64_t)r * 3 * A.N;
    const T *zr = z ? z + (int64_t)r * 3 * A.N : nullptr;
    cpx<T> *sr = spec + (int64_t)r * 3 * A.specN;
    const int64_t p0 = (int64_t)blockIdx.x * pairs_per_block;
    for (int idx = threadIdx.x; idx < pairs_per_block * n0; idx += blockDim.x) {
        const int lp = idx / n0, x = idx - lp * n0;
        const int64_t pr = p0 + lp;
        T a = 0, b = 0;
        if (pr < npairs) {
            const int64_t o0 = (2 * pr) * n0 + x, o1 = o0 + n0;
            a = fr[o0];
            b = fr[o1];
            if (zr) {
                a -= alpha * zr[o0];
                b -= alpha * zr[o1];
                fr[o0] = a;
                fr[o1] = b;
            }
        }
        sh[lp * lstride + x] = {a, b};
    }
    __syncthreads();
    lds_fft<T, false>(sh, pairs_per_block, lstride, pl, tw);
    for (int idx = threadIdx.x; idx < pairs_per_block * nh; idx += blockDim.x) {
        const int lp = idx / nh, kx = idx - lp * nh;
        const int64_t pr = p0 + lp;
        if (pr < npairs) {
            const cpx<T> Zk = sh[lp * lstride + kx];
            const cpx<T> Zm = sh[lp * lstride + (kx == 0 ? 0 : n0 - kx)];
            const cpx<T> Av = {(T)0.5 * (Zk.x + Zm.x), (T)0.5 * (Zk.y - Zm.y)};
            const cpx<T> Bv = {(T)0.5 * (Zk.y + Zm.y), (T)-0.5 * (Zk.x - Zm.x)};
            sr[(2 * pr) * nhs + kx] = Av;
            sr[(2 * pr + 1) * nhs + kx] = Bv;
        }
    }
    // zeros in the row padding: the rows of the workgroup are written as one
    // contiguous stream of whole cache lines
    const int pad = nhs - nh;
    for (int idx = threadIdx.x; idx < pairs_per_block * 2 * pad; idx += blockDim.x) {
        const int lr = idx / pad, k = idx - lr * pad;
        const int64_t row = 2 * p0 + lr;
        if (row < 2 * npairs) sr[row * nhs + nh + k] = cpx<T>{0, 0};
    }
}

// ---------------------------------------------------------------- y pass
template <typename T, bool INV>
__global__ __launch_bounds__(256) void k_fft_y(FftArgs A, FftPlan pl, const cpx<T> *tw, cpx<T> *spec, int tk) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int r = blockIdx.y;
    if (!active_rhs(A, r)) return;
    const int n1 = A.n1, nh = A.nh, nhs = A.nhs;
    const int lstride = n1 + 1;
    const int ntiles = (nh + tk - 1) / tk;
    const int tile = blockIdx.x % ntiles;
    const int plane = blockIdx.x / ntiles;          // c * n2 + k
    const int kx0 = tile * tk;
    cpx<T> *base = spec + (int64_t)r * 3 * A.specN + (int64_t)plane * n1 * nhs;
    for (int idx = threadIdx.x; idx < tk * n1; idx += blockDim.x) {
        const int kl = idx % tk, yy = idx / tk;
        const int kx = kx0 + kl;
        sh[kl * lstride + yy] = (kx < nh) ? base[(int64_t)yy * nhs + kx] : cpx<T>{0, 0};
    }
    __syncthreads();
    lds_fft<T, INV>(sh, tk, lstride, pl, tw);
    for (int idx = threadIdx.x; idx < tk * n1; idx += blockDim.x) {
        const int kl = idx % tk, yy = idx / tk;
        const int kx = kx0 + kl;
        if (kx < nh) base[(int64_t)yy * nhs + kx] = sh[kl * lstride + yy];
    }
}

// ---------------------------------------------------------------- z pass with Green multiply
template <typename T>
__device__ __forceinline__ void green_apply(T s0, T c0, T s1, T c1, T s2, T c2, cpx<T> (&f)[3], bool zero) {
    // half-angle sines/cosines per axis -> symbol entries
    const T q0 = s0 * s0, q1 = s1 * s1, q2 = s2 * s2;
    const T sum = q0 + q1 + q2;
    const T S00 = (T)2 * sum + (T)2 * q0, S11 = (T)2 * sum + (T)2 * q1, S22 = (T)2 * sum + (T)2 * q2;
    // cos(theta) = 1 - 2 s^2, sin(theta) = 2 s c; cos(phi_ab) with phi_ab = half-angle sum
    const T ct0 = (T)1 - (T)2 * q0, st0 = (T)2 * s0 * c0;
    const T ct1 = (T)1 - (T)2 * q1, st1 = (T)2 * s1 * c1;
    const T ct2 = (T)1 - (T)2 * q2, st2 = (T)2 * s2 * c2;
    const T cp01 = c0 * c1 - s0 * s1, sp01 = s0 * c1 + c0 * s1;
    const T cp02 = c0 * c2 - s0 * s2, sp02 = s0 * c2 + c0 * s2;
    const T cp12 = c1 * c2 - s1 * s2, sp12 = s1 * c2 + c1 * s2;
    const T k23 = (T)(2.0 / 3.0);
    const T S01 = k23 * s0 * s1 * ((T)2 * cp01 + (cp01 * ct2 - sp01 * st2));
    const T S02 = k23 * s0 * s2 * ((T)2 * cp02 + (cp02 * ct1 - sp02 * st1));
    const T S12 = k23 * s1 * s2 * ((T)2 * cp12 + (cp12 * ct0 - sp12 * st0));
    // inverse of the symmetric 3x3 matrix by its adjugate
    const T A00 = S11 * S22 - S12 * S12, A01 = S02 * S12 - S01 * S22, A02 = S01 * S12 - S02 * S11;
    const T A11 = S00 * S22 - S02 * S02, A12 = S01 * S02 - S00 * S12, A22 = S00 * S11 - S01 * S01;
    const T det = S00 * A00 + S01 * A01 + S02 * A02;
    const T inv = zero ? (T)0 : (T)1 / det;
    cpx<T> y[3];
    y[0] = {inv * (A00 * f[0].x + A01 * f[1].x + A02 * f[2].x), inv * (A00 * f[0].y + A01 * f[1].y + A02 * f[2].y)};
    y[1] = {inv * (A01 * f[0].x + A11 * f[1].x + A12 * f[2].x), inv * (A01 * f[0].y + A11 * f[1].y + A12 * f[2].y)};
    y[2] = {inv * (A02 * f[0].x + A12 * f[1].x + A22 * f[2].x), inv * (A02 * f[0].y + A12 * f[1].y + A22 * f[2].y)};
    f[0] = y[0];
    f[1] = y[1];
    f[2] = y[2];
}

template <typename T>
__global__ __launch_bounds__(512) void k_fft_z_green(FftArgs A, FftPlan pl, const cpx<T> *tw, const T *h0,
                                                      const T *h1, const T *h2, cpx<T> *spec, int tk, int64_t sz,
                                                      int64_t sy) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    __shared__ double red[8];
    const int n1 = A.n1, n2 = A.n2, nh = A.nh;
    const int lstride = n2 + 1;
    const int ntiles = (nh + tk - 1) / tk;
    const int nblk = n1 * ntiles;                   // workgroups per right-hand side
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(lb / nblk), blk = (int)(lb % nblk);
    if (!active_rhs(A, r)) return;
    const int tile = blk % ntiles;
    const int ky = blk / ntiles;
    const int kx0 = tile * tk;
    cpx<T> *base = spec + (int64_t)r * 3 * A.specN;
    for (int idx = threadIdx.x; idx < 3 * tk * n2; idx += blockDim.x) {
        const int kl = idx % tk, rest = idx / tk;
        const int zz = rest % n2, c = rest / n2;
        const int kx = kx0 + kl;
        sh[(c * tk + kl) * lstride + zz] =
            (kx < nh) ? base[(int64_t)c * A.specN + zz * sz + (int64_t)ky * sy + kx] : cpx<T>{0, 0};
    }
    __syncthreads();
    lds_fft<T, false>(sh, 3 * tk, lstride, pl, tw);
    double part = 0.0;
    const T scale = (T)(1.0 / ((double)A.n0 * (double)n1 * (double)n2));
    for (int idx = threadIdx.x; idx < tk * n2; idx += blockDim.x) {
        const int kl = idx % tk, zz = idx / tk;
        const int kx = kx0 + kl;
        if (kx < nh) {
            cpx<T> f[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = sh[(c * tk + kl) * lstride + zz];
            const cpx<T> f0[3] = {f[0], f[1], f[2]};
            green_apply<T>(h0[2 * kx], h0[2 * kx + 1], h1[2 * ky], h1[2 * ky + 1], h2[2 * zz], h2[2 * zz + 1], f,
                           kx == 0 && ky == 0 && zz == 0);
            double q = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                f[c].x *= scale;
                f[c].y *= scale;
                q += (double)f0[c].x * (double)f[c].x + (double)f0[c].y * (double)f[c].y;
                sh[(c * tk + kl) * lstride + zz] = f[c];
            }
            const double wgt = (kx == 0 || 2 * kx == A.n0) ? 1.0 : 2.0;
            part += wgt * q;
        }
    }
    __syncthreads();
    lds_fft<T, true>(sh, 3 * tk, lstride, pl, tw);
    for (int idx = threadIdx.x; idx < 3 * tk * n2; idx += blockDim.x) {
        const int kl = idx % tk, rest = idx / tk;
        const int zz = rest % n2, c = rest / n2;
        const int kx = kx0 + kl;
        if (kx < nh) base[(int64_t)c * A.specN + zz * sz + (int64_t)ky * sy + kx] = sh[(c * tk + kl) * lstride + zz];
    }
    double v[1] = {part};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) {
        double *P = A.partial + ((int64_t)r * A.nslots + A.slot0 + blk) * NPART;
        P[0] = v[0];
#pragma unroll
        for (int q = 1; q < 7; ++q) P[q] = 0.0;
    }
}

// ---------------------------------------------------------------- x inverse (c2r) + CG update
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_inv(FftArgs A, FftPlan pl, const cpx<T> *tw, const cpx<T> *spec,
                                                    int mode, T *out, T *u, T *d, int pairs_per_block) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int r = blockIdx.y;
    if (!active_rhs(A, r)) return;
    const int n0 = A.n0, nh = A.nh, nhs = A.nhs;
    const int lstride = n0 + 1;
    const int64_t npairs = (int64_t)3 * A.n2 * A.n1 / 2;
    const cpx<T> *sr = spec + (int64_t)r * 3 * A.specN;
    const int64_t p0 = (int64_t)blockIdx.x * pairs_per_block;
    for (int idx = threadIdx.x; idx < pairs_per_block * n0; idx += blockDim.x) {
        const int lp = idx / n0, k = idx - lp * n0;
        const int64_t pr = p0 + lp;
        cpx<T> Zv = {0, 0};
        if (pr < npairs) {
            const bool lo = k < nh;
            const int kk = lo ? k : n0 - k;
            cpx<T> Av = sr[(2 * pr) * nhs + kk], Bv = sr[(2 * pr + 1) * nhs + kk];
            if (!lo) { Av.y = -Av.y; Bv.y = -Bv.y; }
            Zv = {Av.x - Bv.y, Av.y + Bv.x};
        }
        sh[lp * lstride + k] = Zv;
    }
    __syncthreads();
    lds_fft<T, true>(sh, pairs_per_block, lstride, pl, tw);
    const int64_t rN = (int64_t)r * 3 * A.N;
    T alpha = 0, beta = 0;
    if (mode == 1) { alpha = (T)A.scal[r].alpha; beta = (T)A.scal[r].beta; }
    for (int idx = threadIdx.x; idx < pairs_per_block * n0; idx += blockDim.x) {
        const int lp = idx / n0, x = idx - lp * n0;
        const int64_t pr = p0 + lp;
        if (pr < npairs) {
            const cpx<T> yv = sh[lp * lstride + x];
            const int64_t o0 = rN + (2 * pr) * n0 + x, o1 = o0 + n0;
            if (mode == 0) {
                out[o0] = yv.x;
                out[o1] = yv.y;
            } else if (mode == 1) {
                const T d0 = d[o0], d1 = d[o1];
                u[o0] += alpha * d0;
                u[o1] += alpha * d1;
                d[o0] = yv.x + beta * d0;
                d[o1] = yv.y + beta * d1;
            } else {
                d[o0] = yv.x;
                d[o1] = yv.y;
            }
        }
    }
}

// ---------------------------------------------------------------- x and y passes, compile-time length
// Used when the xy plane does not fit in LDS (e.g. 256^2): the x transform on
// PP row pairs per workgroup, the y transform on runs of kx columns; both with
// the LDS Stockham transform of fft_lines.h.  Spectrum layout [c][kz][ky][kx].
template <int N> struct XCfg {
    static constexpr int NH = N / 2 + 1;
    static constexpr int PP = (N >= 256 ? 2048 : 4096) / N;   // row pairs per workgroup
    static constexpr int LS = fft_ls(N);
};

template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft_x_fwd_t(FftArgs A, const cpx<T> *tw, T *f, const T *z, cpx<T> *spec,
                                                      int nrhs) {
    using C = XCfg<N>;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int64_t npairs = (int64_t)3 * A.n2 * A.n1 / 2;
    const int nblk = (int)((npairs + C::PP - 1) / C::PP);
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(lb / nblk), blk = (int)(lb % nblk);
    if (!active_rhs(A, r)) return;
    const T alpha = z ? (T)A.scal[r].alpha : (T)0;
    T *fr = f + (int64_t)r * 3 * A.N;
    const T *zr = z ? z + (int64_t)r * 3 * A.N : nullptr;
    cpx<T> *sr = spec + (int64_t)r * 3 * A.specN;
    const int64_t p0 = (int64_t)blk * C::PP;
    for (int idx = threadIdx.x; idx < C::PP * N; idx += 256) {
        const int lp = idx / N, x = idx - lp * N;
        const int64_t pr = p0 + lp;
        T a = 0, b = 0;
        if (pr < npairs) {
            const int64_t o0 = (2 * pr) * N + x, o1 = o0 + N;
            a = fr[o0];
            b = fr[o1];
            if (zr) {
                a -= alpha * zr[o0];
                b -= alpha * zr[o1];
                fr[o0] = a;
                fr[o1] = b;
            }
        }
        sh[lp * C::LS + fft_pad(x)] = {a, b};
    }
    __syncthreads();
    fft_lines<T, N, C::PP, 256, false>(sh, tw);
    for (int idx = threadIdx.x; idx < C::PP * C::NH; idx += 256) {
        const int lp = idx / C::NH, kx = idx - lp * C::NH;
        const int64_t pr = p0 + lp;
        if (pr < npairs) {
            const cpx<T> Zk = sh[lp * C::LS + fft_pad(kx)];
            const cpx<T> Zm = sh[lp * C::LS + fft_pad(kx == 0 ? 0 : N - kx)];
            sr[(2 * pr) * A.nhs + kx] = {(T)0.5 * (Zk.x + Zm.x), (T)0.5 * (Zk.y - Zm.y)};
            sr[(2 * pr + 1) * A.nhs + kx] = {(T)0.5 * (Zk.y + Zm.y), (T)-0.5 * (Zk.x - Zm.x)};
        }
    }
    // zeros in the row padding: the rows of the workgroup are written as one
    // contiguous stream of whole cache lines
    const int pad = A.nhs - C::NH;
    for (int idx = threadIdx.x; idx < C::PP * 2 * pad; idx += 256) {
        const int lr = idx / pad, k = idx - lr * pad;
        const int64_t row = 2 * p0 + lr;
        if (row < 2 * npairs) sr[row * A.nhs + C::NH + k] = cpx<T>{0, 0};
    }
}

// mode 0: out = G f; mode 1: u += alpha d, d = G f + beta d; mode 2: d = G f
template <typename T, int N>
__global__ __launch_bounds__(256) void k_fft_x_inv_t(FftArgs A, const cpx<T> *tw, const cpx<T> *spec, int mode,
                                                      T *out, T *u, T *d, int nrhs) {
    using C = XCfg<N>;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int64_t npairs = (int64_t)3 * A.n2 * A.n1 / 2;
    const int nblk = (int)((npairs + C::PP - 1) / C::PP);
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(lb / nblk), blk = (int)(lb % nblk);
    if (!active_rhs(A, r)) return;
    const cpx<T> *sr = spec + (int64_t)r * 3 * A.specN;
    const int64_t p0 = (int64_t)blk * C::PP;
    for (int idx = threadIdx.x; idx < C::PP * N; idx += 256) {
        const int lp = idx / N, k = idx - lp * N;
        const int64_t pr = p0 + lp;
        cpx<T> Zv = {0, 0};
        if (pr < npairs) {
            const bool lo = k < C::NH;
            const int kk = lo ? k : N - k;
            cpx<T> Av = sr[(2 * pr) * A.nhs + kk], Bv = sr[(2 * pr + 1) * A.nhs + kk];
            if (!lo) { Av.y = -Av.y; Bv.y = -Bv.y; }
            Zv = {Av.x - Bv.y, Av.y + Bv.x};
        }
        sh[lp * C::LS + fft_pad(k)] = Zv;
    }
    __syncthreads();
    fft_lines<T, N, C::PP, 256, true>(sh, tw);
    const int64_t rN = (int64_t)r * 3 * A.N;
    T alpha = 0, beta = 0;
    if (mode == 1) { alpha = (T)A.scal[r].alpha; beta = (T)A.scal[r].beta; }
    for (int idx = threadIdx.x; idx < C::PP * N; idx += 256) {
        const int lp = idx / N, x = idx - lp * N;
        const int64_t pr = p0 + lp;
        if (pr < npairs) {
            const cpx<T> yv = sh[lp * C::LS + fft_pad(x)];
            const int64_t o0 = rN + (2 * pr) * N + x, o1 = o0 + N;
            if (mode == 0) {
                out[o0] = yv.x;
                out[o1] = yv.y;
            } else if (mode == 1) {
                const T d0 = d[o0], d1 = d[o1];
                u[o0] += alpha * d0;
                u[o1] += alpha * d1;
                d[o0] = yv.x + beta * d0;
                d[o1] = yv.y + beta * d1;
            } else {
                d[o0] = yv.x;
                d[o1] = yv.y;
            }
        }
    }
}

// y transform of runs of up to TK kx columns of one (component, kz) plane; the
// ceil(nh / TK) runs share the nh columns evenly
template <typename T, int N1, int TK, bool INV>
__global__ __launch_bounds__(256) void k_fft_y_t(FftArgs A, const cpx<T> *tw, cpx<T> *spec, int nrhs) {
    constexpr int LS = fft_ls(N1);
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int nh = A.nh;
    const int ntiles = (nh + TK - 1) / TK;
    const int tk = (nh + ntiles - 1) / ntiles;
    const int nblk = 3 * A.n2 * ntiles;
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(lb / nblk), blk = (int)(lb % nblk);
    if (!active_rhs(A, r)) return;
    const int tile = blk % ntiles, plane = blk / ntiles;       // plane = c * n2 + kz
    const int kx0 = tile * tk, ncol = min(tk, nh - kx0);
    cpx<T> *base = spec + (int64_t)r * 3 * A.specN + (int64_t)plane * N1 * A.nhs + kx0;
    for (int idx = threadIdx.x; idx < TK * N1; idx += 256) {
        const int kl = idx % TK, yy = idx / TK;
        if (kl < tk) sh[kl * LS + fft_pad(yy)] = kl < ncol ? base[(int64_t)yy * A.nhs + kl] : cpx<T>{0, 0};
    }
    __syncthreads();
    fft_lines<T, N1, TK, 256, INV>(sh, tw, tk);
    for (int idx = threadIdx.x; idx < TK * N1; idx += 256) {
        const int kl = idx % TK, yy = idx / TK;
        if (kl < ncol) base[(int64_t)yy * A.nhs + kl] = sh[kl * LS + fft_pad(yy)];
    }
}

// ---------------------------------------------------------------- xy plane kernels (n0 == n1 == N)
// A workgroup transforms one (component, z plane, load) plane held in LDS:
// the x transform runs on row pairs packed as complex lines, the y transform on
// the kx columns.  Spectrum layout [c][ky][kz][kx] (kx fastest).  In FP32 the
// kernels need at most 64 registers, so two 1024-thread workgroups share a CU
// and one's loads and stores overlap the other's transform.  LDS uses the interleaved layout of fft_lines.h (line l at l * (N | 1), no
// padding), so the transposes between the x and y transforms, which address
// 32 consecutive lines at one offset or one line at 32 consecutive offsets,
// are conflict free as well.
template <int N> struct PlaneCfg {
    static constexpr int NH = N / 2 + 1;
    static constexpr int NP = N / 2;
    static constexpr int LS = lds_ls<true>(N);
    static constexpr int NT = 1024;
    static constexpr int ELEMS = NH * LS;      // >= NP * LS
    static constexpr int NIN = NP * N;         // packed row-pair elements of a plane
    static constexpr int PE = (NIN + NT - 1) / NT;
    static constexpr int NSP = N * NH;         // half-spectrum elements of a plane
    static constexpr int PS = (NSP + NT - 1) / NT;
    // N = 64, 128: thread (kxl, kyl) = (tid % KW, tid / KW) handles columns
    // kx = kxl < KW at rows kyl + RS m (the Nyquist column kx = KW by threads
    // tid < N), so that all LDS offsets are per-thread bases plus compile-time
    // constants and no index is divided by NH
    static constexpr int KW = N / 2;
    static constexpr int RS = NT / KW;
    static constexpr bool FP = (N == 64 || N == 128);
    static constexpr int SW = FP ? N / RS : 1;     // spectrum sweeps per plane
    static constexpr int XW = FP ? NP / RS : 1;    // split sweeps per plane
};

// LDS holds the packed row pairs of a plane: x transform, split into the two
// real rows' spectra, transpose to kx-major lines, y transform, store.
template <typename T, int N>
__device__ __forceinline__ void plane_forward_core(cpx<T> *sh, const cpx<T> *tw, const FftArgs &A, cpx<T> *sr,
                                                   int kz, int tid) {
    using C = PlaneCfg<N>;
    fft_lines<T, N, C::NP, C::NT, false, true>(sh, tw, C::NP, tid);
    if constexpr (C::FP) {
        const int kxl = tid % C::KW, ppl = tid / C::KW;
        const int rd = ppl * C::LS + kxl, rdm = ppl * C::LS + (kxl == 0 ? 0 : N - kxl);
        cpx<T> ra[C::XW + 1], rb[C::XW + 1];
#pragma unroll
        for (int m = 0; m < C::XW; ++m) {
            const cpx<T> Zk = sh[rd + m * C::RS * C::LS], Zm = sh[rdm + m * C::RS * C::LS];
            ra[m] = {(T)0.5 * (Zk.x + Zm.x), (T)0.5 * (Zk.y - Zm.y)};
            rb[m] = {(T)0.5 * (Zk.y + Zm.y), (T)-0.5 * (Zk.x - Zm.x)};
        }
        if (tid < C::NP) {                 // Nyquist column kx = KW of row pair tid
            const cpx<T> Zk = sh[tid * C::LS + C::KW];
            ra[C::XW] = {(T)0.5 * (Zk.x + Zk.x), (T)0.5 * (Zk.y - Zk.y)};
            rb[C::XW] = {(T)0.5 * (Zk.y + Zk.y), (T)-0.5 * (Zk.x - Zk.x)};
        }
        __syncthreads();
        const int wr = kxl * C::LS + 2 * ppl, wr1 = kxl * C::LS + 2 * ppl + 1;
#pragma unroll
        for (int m = 0; m < C::XW; ++m) {
            constexpr int step = 2 * C::RS;
            sh[wr + m * step] = ra[m];
            sh[wr1 + m * step] = rb[m];
        }
        if (tid < C::NP) {
            sh[C::KW * C::LS + 2 * tid] = ra[C::XW];
            sh[C::KW * C::LS + 2 * tid + 1] = rb[C::XW];
        }
        __syncthreads();
        fft_lines<T, N, C::NH, C::NT, false, true>(sh, tw, C::NH, tid);
        // spectrum rows ky = kyl + RS m of columns kxl, and the Nyquist column
        const int kyl = ppl;
        cpx<T> *so = sr + ((int64_t)kyl * A.n2 + kz) * C::NH + kxl;
        const int64_t sstep = (int64_t)C::RS * A.n2 * C::NH;
        const int ld = kxl * C::LS + kyl;
#pragma unroll
        for (int m = 0; m < C::SW; ++m) so[m * sstep] = sh[ld + m * C::RS];
        if (tid < N) sr[((int64_t)tid * A.n2 + kz) * C::NH + C::KW] = sh[C::KW * C::LS + tid];
        return;
    }
    constexpr int NOUT = C::NP * C::NH;
    constexpr int MO = (NOUT + C::NT - 1) / C::NT;
    cpx<T> ra[MO], rb[MO];
#pragma unroll
    for (int i = 0; i < MO; ++i) {
        const int idx = tid + i * C::NT;
        if (idx < NOUT) {
            const int pp = idx / C::NH, kx = idx - pp * C::NH;
            const cpx<T> Zk = sh[pp * C::LS + kx];
            const cpx<T> Zm = sh[pp * C::LS + (kx == 0 ? 0 : N - kx)];
            ra[i] = {(T)0.5 * (Zk.x + Zm.x), (T)0.5 * (Zk.y - Zm.y)};
            rb[i] = {(T)0.5 * (Zk.y + Zm.y), (T)-0.5 * (Zk.x - Zm.x)};
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MO; ++i) {
        const int idx = tid + i * C::NT;
        if (idx < NOUT) {
            const int pp = idx / C::NH, kx = idx - pp * C::NH;
            sh[kx * C::LS + 2 * pp] = ra[i];
            sh[kx * C::LS + 2 * pp + 1] = rb[i];
        }
    }
    __syncthreads();
    fft_lines<T, N, C::NH, C::NT, false, true>(sh, tw, C::NH, tid);
    for (int idx = tid; idx < N * C::NH; idx += C::NT) {
        const int ky = idx / C::NH, kx = idx - ky * C::NH;
        sr[((int64_t)ky * A.n2 + kz) * C::NH + kx] = sh[kx * C::LS + ky];
    }
}

template <typename T, int N>
__global__ __launch_bounds__(1024) void k_fft_plane_fwd(FftArgs A, const cpx<T> *tw, T *f, const T *z,
                                                         cpx<T> *spec, int nrhs) {
    using C = PlaneCfg<N>;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    const int per_r = 3 * A.n2;
    const int q = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int r = q / per_r, plane = q - r * per_r;
    if (!active_rhs(A, r)) return;
    const int c = plane / A.n2, kz = plane - c * A.n2;
    int tid = threadIdx.x;
    // opaque to the optimiser: the index arithmetic of each phase is recomputed
    // from tid instead of being kept live across the transform (fewer registers)
    asm volatile("" : "+v"(tid));
    T *fr = f + (int64_t)r * 3 * A.N + (int64_t)plane * N * N;
    const T *zr = z ? z + (int64_t)r * 3 * A.N + (int64_t)plane * N * N : nullptr;
    const T alpha = z ? (T)A.scal[r].alpha : (T)0;
    // fused residual update f -= alpha z; pack row pairs
#pragma unroll
    for (int i = 0; i < C::PE; ++i) {
        const int idx = tid + i * C::NT;
        if (C::NIN % C::NT == 0 || idx < C::NIN) {
            const int pp = idx / N, x = idx - pp * N;
            const int o0 = (2 * pp) * N + x;
            T a = fr[o0], b = fr[o0 + N];
            if (zr) {
                a -= alpha * zr[o0];
                b -= alpha * zr[o0 + N];
                fr[o0] = a;
                fr[o0 + N] = b;
            }
            sh[pp * C::LS + x] = {a, b};
        }
    }
    __syncthreads();
    plane_forward_core<T, N>(sh, tw, A, spec + (int64_t)r * 3 * A.specN + (int64_t)c * A.specN, kz, tid);
}

// LDS holds the kx-major half spectrum of a plane: y inverse transform,
// rebuild the packed row pairs, x inverse transform.
template <typename T, int N>
__device__ __forceinline__ void plane_inverse_core(cpx<T> *sh, const cpx<T> *tw, int tid) {
    using C = PlaneCfg<N>;
    fft_lines<T, N, C::NH, C::NT, true, true>(sh, tw, C::NH, tid);
    if constexpr (C::FP) {
        // output (row pair ppl + RP i, x = k) for thread (k, ppl) = (tid % N, tid / N)
        constexpr int RP = C::NT / N, NI = C::NP / RP;
        const int k = tid % N, ppl = tid / N;
        const bool lo = k < C::NH;
        const int kk = lo ? k : N - k;
        const int ra0 = kk * C::LS + 2 * ppl, rb0 = kk * C::LS + 2 * ppl + 1;
        constexpr int rstep = 2 * RP;
        cpx<T> rz[NI];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            cpx<T> Av = sh[ra0 + i * rstep], Bv = sh[rb0 + i * rstep];
            if (!lo) { Av.y = -Av.y; Bv.y = -Bv.y; }
            rz[i] = {Av.x - Bv.y, Av.y + Bv.x};
        }
        __syncthreads();
        const int w0 = ppl * C::LS + k;
#pragma unroll
        for (int i = 0; i < NI; ++i) sh[w0 + i * RP * C::LS] = rz[i];
        __syncthreads();
        fft_lines<T, N, C::NP, C::NT, true, true>(sh, tw, C::NP, tid);
        return;
    }
    constexpr int NOUT = C::NP * N;
    constexpr int MO = (NOUT + C::NT - 1) / C::NT;
    cpx<T> rz[MO];
#pragma unroll
    for (int i = 0; i < MO; ++i) {
        const int idx = tid + i * C::NT;
        if (idx < NOUT) {
            const int pp = idx / N, k = idx - pp * N;
            const bool lo = k < C::NH;
            const int kk = lo ? k : N - k;
            cpx<T> Av = sh[kk * C::LS + 2 * pp], Bv = sh[kk * C::LS + 2 * pp + 1];
            if (!lo) { Av.y = -Av.y; Bv.y = -Bv.y; }
            rz[i] = {Av.x - Bv.y, Av.y + Bv.x};
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MO; ++i) {
        const int idx = tid + i * C::NT;
        if (idx < NOUT) {
            const int pp = idx / N, k = idx - pp * N;
            sh[pp * C::LS + k] = rz[i];
        }
    }
    __syncthreads();
    fft_lines<T, N, C::NP, C::NT, true, true>(sh, tw, C::NP, tid);
}

// mode 0: out = G f; mode 1: u += alpha d, d = G f + beta d; mode 2: d = G f
template <typename T, int N>
__global__ __launch_bounds__(1024) void k_fft_plane_inv(FftArgs A, const cpx<T> *tw, const cpx<T> *spec, int mode,
                                                         T *out, T *u, T *d, int nrhs, EnrFin<T> E) {
    using C = PlaneCfg<N>;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    int tid = threadIdx.x;
    if (E.mode) {
        // enriched direction update, spread over the whole grid
        for (int r = 0; r < nrhs; ++r)
            if (active_rhs(A, r))
                enr_final_rows<T>(E, A.scal, r, (int64_t)blockIdx.x * C::NT + tid, (int64_t)gridDim.x * C::NT);
    }
    const int per_r = 3 * A.n2;
    const int q = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int r = q / per_r, plane = q - r * per_r;
    if (!active_rhs(A, r)) return;
    const int c = plane / A.n2, kz = plane - c * A.n2;
    // opaque to the optimiser: index arithmetic is recomputed per phase (fewer registers)
    asm volatile("" : "+v"(tid));
    const cpx<T> *sr = spec + (int64_t)r * 3 * A.specN + (int64_t)c * A.specN;
    if constexpr (C::FP) {
        const int kxl = tid % C::KW, kyl = tid / C::KW;
        const cpx<T> *si = sr + ((int64_t)kyl * A.n2 + kz) * C::NH + kxl;
        const int64_t sstep = (int64_t)C::RS * A.n2 * C::NH;
        const int st = kxl * C::LS + kyl;
#pragma unroll
        for (int m = 0; m < C::SW; ++m) sh[st + m * C::RS] = si[m * sstep];
        if (tid < N) sh[C::KW * C::LS + tid] = sr[((int64_t)tid * A.n2 + kz) * C::NH + C::KW];
    } else {
#pragma unroll
        for (int i = 0; i < C::PS; ++i) {
            const int idx = tid + i * C::NT;
            if (C::NSP % C::NT == 0 || idx < C::NSP) {
                const int ky = idx / C::NH, kx = idx - ky * C::NH;
                sh[kx * C::LS + ky] = sr[((int64_t)ky * A.n2 + kz) * C::NH + kx];
            }
        }
    }
    __syncthreads();
    plane_inverse_core<T, N>(sh, tw, tid);
    const int64_t base = (int64_t)r * 3 * A.N + (int64_t)plane * N * N;
    T alpha = 0, beta = 0;
    if (mode == 1) { alpha = (T)A.scal[r].alpha; beta = (T)A.scal[r].beta; }
#pragma unroll
    for (int i = 0; i < C::PE; ++i) {
        const int idx = tid + i * C::NT;
        if (C::NIN % C::NT == 0 || idx < C::NIN) {
            const int pp = idx / N, x = idx - pp * N;
            const cpx<T> yv = sh[pp * C::LS + x];
            const int64_t o0 = base + (unsigned)((2 * pp) * N + x), o1 = o0 + N;
            if (mode == 0) {
                out[o0] = yv.x;
                out[o1] = yv.y;
            } else if (mode == 1) {
                const T d0 = d[o0], d1 = d[o1];
                u[o0] += alpha * d0;
                u[o1] += alpha * d1;
                d[o0] = yv.x + beta * d0;
                d[o1] = yv.y + beta * d1;
            } else {
                d[o0] = yv.x;
                d[o1] = yv.y;
            }
        }
    }
}

// ---------------------------------------------------------------- z pass, compile-time length
// Element (c, kz, ky, kx) of the spectrum at c * specN + kz * sz + ky * sy + kx.
// One workgroup per (ky, run of tk kx columns, load); the ceil(nh / TK) runs
// share the nh columns evenly (tk <= TK), so no run is mostly padding.  LDS
// line c * tk + kl holds component c of column kx0 + kl.  Workgroups of the
// active loads are numbered so that every XCD takes one contiguous range
// (neighbouring runs share cache lines).  Thread (kl, z0) = (tid % TK, tid / TK)
// handles column kl at rows z0 + m ZR (ZR = 512 / TK): when ZR divides n2 all
// global and LDS offsets of its elements are compile-time constants added to
// three per-thread bases.  With 3 TK >= 32 lines the LDS uses the interleaved
// layout of fft_lines.h; the two row groups of a half wave then sit ZR / 2
// rows apart, so that the 16 columns x 2 rows of a half wave fall on 32
// different banks in the staging and Green phases too.
template <typename T, int N2, int TK>
// FP32 tiles of up to 2048 staged values per component are held to 64
// registers (eight waves per SIMD); larger tiles fit one workgroup per CU in
// LDS, so they keep their registers
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && TK * N2 <= 2048 ? 8 : 1)))
void k_fft_z_t(FftArgs A, const cpx<T> *tw, const T *h0, const T *h1,
                                                  const T *h2, cpx<T> *spec, int64_t sz, int64_t sy, int nrhs,
                                                  EnrUpd<T> E) {
    static_assert(ENR_BLOCK == 512, "the enriched workgroups use the z-pass workgroup size");
    constexpr int NL = 3 * TK;
    constexpr bool ILV = NL >= 32;
    constexpr int LS = lds_ls<ILV>(N2);
    constexpr int NE = NL * N2;                     // staged elements of a workgroup
    static_assert(512 % TK == 0, "TK must divide the workgroup");
    constexpr int ZR = 512 / TK;
    constexpr bool FAST = N2 % ZR == 0 && ZR % 16 == 0;
    extern __shared__ unsigned char smem_raw[];
    cpx<T> *sh = reinterpret_cast<cpx<T> *>(smem_raw);
    __shared__ double red[8];
    const int nh = A.nh;
    const int ntiles = (nh + TK - 1) / TK;
    const int nblk = A.n1 * ntiles;                 // workgroups per right-hand side
    const int tk = (nh + ntiles - 1) / ntiles;
    if ((int)blockIdx.x >= nblk * nrhs) {
        // enriched residual update (workgroups after the z-pass ones)
        const int e = (int)blockIdx.x - nblk * nrhs, re = e / E.nblk;
        if (active_rhs(A, re)) enr_update_block<T>(E, A.scal, A.partial, A.nslots, re, e - re * E.nblk, red);
        return;
    }
    int nact = 0;
    for (int q = 0; q < nrhs; ++q) nact += active_rhs(A, q) ? 1 : 0;
    const int total = nact * nblk;
    if ((int)blockIdx.x >= total) return;
    const int L = (int)xcd_remap(blockIdx.x, total);
    int ka = L / nblk;
    const int blk = L - ka * nblk;
    int r = 0;
    while (!active_rhs(A, r) || ka-- > 0) ++r;      // the ka-th active load
    const int tile = blk % ntiles, ky = blk / ntiles;
    const int kx0 = tile * tk, ncol = min(tk, nh - kx0);
    cpx<T> *base = spec + (int64_t)r * 3 * A.specN + (int64_t)ky * sy + kx0;
    const int tid = threadIdx.x;
    const int kl = tid % TK, q = tid / TK;
    const int z0 = (ILV && TK == 16 && ZR % 2 == 0) ? (q >> 1) + (ZR / 2) * (q & 1) : q;
    const T scale = (T)(1.0 / ((double)A.n0 * (double)A.n1 * (double)N2));
    double part = 0.0;
    if constexpr (FAST) {
        constexpr int NSW = 3 * N2 / ZR;            // sweeps over (component, row)
        constexpr int NZ = N2 / ZR;                 // rows per thread and component
        cpx<T> *gb = base + kl + (int64_t)z0 * sz;
        int lb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) lb[c] = (c * tk + kl) * LS + lds_pos<ILV>(z0);
        if (kl < tk) {
#pragma unroll
            for (int m = 0; m < NSW; ++m) {
                const int c = (m * ZR) / N2, zo = (m * ZR) % N2;
                sh[lb[c] + lds_pos<ILV>(zo)] = kl < ncol ? gb[(int64_t)c * A.specN + (int64_t)zo * sz] : cpx<T>{0, 0};
            }
        }
        __syncthreads();
        fft_lines<T, N2, NL, 512, false, ILV>(sh, tw, 3 * tk, tid);
        if (kl < ncol) {
            const int kx = kx0 + kl;
            const T s0 = h0[2 * kx], c0 = h0[2 * kx + 1], s1 = h1[2 * ky], c1 = h1[2 * ky + 1];
            const double wk = (kx == 0 || 2 * kx == A.n0) ? 1.0 : 2.0;
#pragma unroll
            for (int m = 0; m < NZ; ++m) {
                const int zz = z0 + m * ZR, off = lds_pos<ILV>(m * ZR);
                cpx<T> fv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) fv[c] = sh[lb[c] + off];
                const cpx<T> f0[3] = {fv[0], fv[1], fv[2]};
                green_apply<T>(s0, c0, s1, c1, h2[2 * zz], h2[2 * zz + 1], fv, kx == 0 && ky == 0 && zz == 0);
                double q = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    fv[c].x *= scale;
                    fv[c].y *= scale;
                    q += (double)f0[c].x * (double)fv[c].x + (double)f0[c].y * (double)fv[c].y;
                    sh[lb[c] + off] = fv[c];
                }
                part += wk * q;
            }
        }
        __syncthreads();
        fft_lines<T, N2, NL, 512, true, ILV>(sh, tw, 3 * tk, tid);
        if (kl < ncol) {
#pragma unroll
            for (int m = 0; m < NSW; ++m) {
                const int c = (m * ZR) / N2, zo = (m * ZR) % N2;
                gb[(int64_t)c * A.specN + (int64_t)zo * sz] = sh[lb[c] + lds_pos<ILV>(zo)];
            }
        }
    } else {
        for (int idx = tid; idx < NE; idx += 512) {
            const int k = idx % TK, rest = idx / TK;
            const int zz = rest % N2, c = rest / N2;
            if (k < tk)
                sh[(c * tk + k) * LS + lds_pos<ILV>(zz)] = k < ncol ? base[(int64_t)c * A.specN + zz * sz + k] : cpx<T>{0, 0};
        }
        __syncthreads();
        fft_lines<T, N2, NL, 512, false, ILV>(sh, tw, 3 * tk, tid);
        for (int idx = tid; idx < TK * N2; idx += 512) {
            const int k = idx % TK, zz = idx / TK;
            const int kx = kx0 + k;
            if (k < ncol) {
                cpx<T> fv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) fv[c] = sh[(c * tk + k) * LS + lds_pos<ILV>(zz)];
                const cpx<T> f0[3] = {fv[0], fv[1], fv[2]};
                green_apply<T>(h0[2 * kx], h0[2 * kx + 1], h1[2 * ky], h1[2 * ky + 1], h2[2 * zz], h2[2 * zz + 1],
                               fv, kx == 0 && ky == 0 && zz == 0);
                double q = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    fv[c].x *= scale;
                    fv[c].y *= scale;
                    q += (double)f0[c].x * (double)fv[c].x + (double)f0[c].y * (double)fv[c].y;
                    sh[(c * tk + k) * LS + lds_pos<ILV>(zz)] = fv[c];
                }
                part += ((kx == 0 || 2 * kx == A.n0) ? 1.0 : 2.0) * q;
            }
        }
        __syncthreads();
        fft_lines<T, N2, NL, 512, true, ILV>(sh, tw, 3 * tk, tid);
        for (int idx = tid; idx < NE; idx += 512) {
            const int k = idx % TK, rest = idx / TK;
            const int zz = rest % N2, c = rest / N2;
            if (k < ncol) base[(int64_t)c * A.specN + zz * sz + k] = sh[(c * tk + k) * LS + lds_pos<ILV>(zz)];
        }
    }
    double pv[1] = {part};
    block_sum<1>(pv, red);
    if (tid == 0) {
        double *P = A.partial + ((int64_t)r * A.nslots + A.slot0 + blk) * NPART;
        P[0] = pv[0];
#pragma unroll
        for (int q = 1; q < 7; ++q) P[q] = 0.0;
    }
}

template <typename T> int pairs_for(int n0) {
    // limit: butterflies per stage <= MAXB * 256 (radix 2 worst case) and LDS <= 64 KiB
    int p = (MAXB * 256 * 2) / n0;
    const int lds_cap = (int)(65536 / ((n0 + 1) * sizeof(cpx<T>)));
    if (p > lds_cap) p = lds_cap;
    if (p < 1) p = 1;
    return p;
}
template <typename T> int tk_for(int n, int lines_factor, int threads) {
    int t = (MAXB * threads * 2) / (n * lines_factor);
    const int lds_cap = (int)(65536 / ((n + 1) * sizeof(cpx<T>) * lines_factor));
    if (t > lds_cap) t = lds_cap;
    if (t > 16) t = 16;
    if (t < 1) t = 1;
    return t;
}

template <typename T>
FftArgs fft_args(xfft_problem *p, const Flags *flags, int parity) {
    FftArgs A;
    A.n0 = p->g.n0; A.n1 = p->g.n1; A.n2 = p->g.n2; A.nh = p->g.nh; A.nhs = p->g.nh;
    A.N = p->g.N;
    A.specN = (int64_t)p->g.n2 * p->g.n1 * p->g.nh;
    A.flags = flags; A.parity = parity; A.scal = p->scal;
    A.partial = p->partial; A.nslots = p->nslots; A.slot0 = 0;
    return A;
}

}  // namespace

// The generic z pass (runtime line length) uses the FP64 tile width in both precisions.
static int tk_z(const Geometry &g) { return tk_for<double>(g.n2, 3, 512); }

static bool plane_size(int n) { return n == 16 || n == 32 || n == 48 || n == 64 || n == 96 || n == 128; }
static bool ztmpl_size(int n) { return plane_size(n) || n == 256; }

template <typename T> static bool plane_path(const Geometry &g) {
    return g.n0 == g.n1 && plane_size(g.n0) &&
           (size_t)(g.n0 / 2 + 1) * lds_ls<true>(g.n0) * sizeof(cpx<T>) <= (size_t)160 * 1024;
}
// the xy-plane kernels run when the grid has them and the problem's variant selects them
template <typename T> static bool use_plane(const xfft_problem *p) {
    return plane_path<T>(p->g) && p->fft_plane[sizeof(T) == 8 ? 1 : 0] != 0;
}
// Spectrum layout of a Green application: the xy-plane kernels keep rows of nh
// values ([c][ky][kz][kx]); the separate passes ([c][kz][ky][kx]) pad the rows to
// a multiple of 8 values, so that the kx runs the y and z passes move start on
// 64-byte (FP32) or 128-byte (FP64) boundaries instead of straddling cache lines.
template <typename T> static void set_spec_layout(const xfft_problem *p, FftArgs &A) {
    A.nhs = use_plane<T>(p) ? p->g.nh : spec_row_stride(p->g.nh);
    A.specN = (int64_t)p->g.n2 * p->g.n1 * A.nhs;
}
// kx columns per z-pass workgroup: 3 x TK lines of n2 complex values in LDS
// (about 50 KB, three workgroups per CU)
template <typename T> static constexpr int tkz_t(int n2) { return (sizeof(T) == 8 ? 8 : 16) / (n2 >= 256 ? 2 : 1); }
// the alternative tile: twice the columns at n2 = 256 (128-byte runs in FP32,
// one or two workgroups per CU), half of them below (more workgroups per CU)
template <typename T> static constexpr int tkz_alt(int n2) { return n2 >= 256 ? 2 * tkz_t<T>(n2) : tkz_t<T>(n2) / 2; }

// The generic passes run every line of a workgroup through lds_fft, which
// handles at most MAXB * threads butterflies per stage, and hold their lines
// in at most 64 KiB of LDS.  A grid whose generic pass would exceed either
// limit is rejected at setup.
static bool ct_xy_size(int n) { return ztmpl_size(n); }
static int min_radix(int n) {
    const FftPlan pl = make_plan(n);
    int r = 4;
    for (int s = 0; s < pl.nstages; ++s) r = pl.radix[s] < r ? pl.radix[s] : r;
    return r;
}
template <typename T> static bool generic_fits(int lines, int n, int threads) {
    return (int64_t)lines * (n / min_radix(n)) <= (int64_t)MAXB * threads &&
           (size_t)lines * (n + 1) * sizeof(cpx<T>) <= (size_t)65536;
}
template <typename T> static bool fft_fits(const Geometry &g) {
    if (!plane_path<T>(g)) {
        if (!ct_xy_size(g.n0) && !generic_fits<T>(pairs_for<T>(g.n0), g.n0, 256)) return false;
        if (!ct_xy_size(g.n1) && !generic_fits<T>(tk_for<T>(g.n1, 1, 256), g.n1, 256)) return false;
    }
    if (!ztmpl_size(g.n2) && !generic_fits<T>(3 * tk_z(g), g.n2, 512)) return false;
    return true;
}
bool fft_sizes_ok(int n0, int n1, int n2) {
    Geometry g{};
    g.n0 = n0; g.n1 = n1; g.n2 = n2; g.nh = n0 / 2 + 1;
    g.N = (int64_t)n0 * n1 * n2;
    for (int n : {n0, n1, n2})
        if (make_plan(n).nstages < 0) return false;
    return fft_fits<double>(g) && fft_fits<float>(g);
}

template <typename T> static int green_blocks_tk(const Geometry &g, int ztile) {
    const int tk = ztmpl_size(g.n2) ? (ztile ? tkz_alt<T>(g.n2) : tkz_t<T>(g.n2)) : tk_z(g);
    return g.n1 * ((g.nh + tk - 1) / tk);
}
template <typename T> int green_blocks(const xfft_problem *p) {
    return green_blocks_tk<T>(p->g, p->fft_ztile[sizeof(T) == 8 ? 1 : 0]);
}
template int green_blocks<double>(const xfft_problem *);
template int green_blocks<float>(const xfft_problem *);

template <typename T> int fft_variants(const Geometry &g) {
    return (plane_path<T>(g) ? 1 : 0) | (ztmpl_size(g.n2) ? 2 : 0);
}
template int fft_variants<double>(const Geometry &);
template int fft_variants<float>(const Geometry &);

// partial-sum slots for the z pass: the most workgroups any variant launches
int green_slots(const Geometry &g) {
    int m = 0;
    for (int zt = 0; zt < 2; ++zt) {
        m = std::max(m, green_blocks_tk<double>(g, zt));
        m = std::max(m, green_blocks_tk<float>(g, zt));
    }
    return m;
}

template <typename K> static void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// one workgroup per (load, component, z plane); two are resident per CU
static unsigned plane_grid(const xfft_problem *p, int nrhs) { return (unsigned)(3 * p->g.n2 * nrhs); }

template <typename T, int N>
static void plane_fwd(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s, const cpx<T> *tw, T *f,
                      const T *z, cpx<T> *spec) {
    const size_t lds = (size_t)PlaneCfg<N>::ELEMS * sizeof(cpx<T>);
    static bool init = false;
    if (!init) { allow_lds(k_fft_plane_fwd<T, N>, lds); init = true; }
    k_fft_plane_fwd<T, N><<<plane_grid(p, nrhs), PlaneCfg<N>::NT, lds, s>>>(A, tw, f, z, spec, nrhs);
}
template <typename T, int N>
static void plane_inv(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s, const cpx<T> *tw,
                      const cpx<T> *spec, int mode, T *out, T *u, T *d, const EnrFin<T> &E) {
    const size_t lds = (size_t)PlaneCfg<N>::ELEMS * sizeof(cpx<T>);
    static bool init = false;
    if (!init) { allow_lds(k_fft_plane_inv<T, N>, lds); init = true; }
    k_fft_plane_inv<T, N><<<plane_grid(p, nrhs), PlaneCfg<N>::NT, lds, s>>>(A, tw, spec, mode, out, u, d, nrhs, E);
}
template <typename T, int N2, int TK>
static void zpass_tk(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s, const Tables<T> &tb, cpx<T> *spec,
                     int64_t sz, int64_t sy, const EnrUpd<T> &E) {
    // LDS holds the 3 tk lines a workgroup uses (tk <= TK columns share the nh
    // columns evenly); at 128^3 in FP32 that is 13 of 16, which lets four
    // workgroups share a CU (64 registers, eight waves per SIMD)
    const int nh = p->g.nh, ntiles = (nh + TK - 1) / TK, tk = (nh + ntiles - 1) / ntiles;
    const size_t line = (size_t)lds_ls<3 * TK >= 32>(N2) * sizeof(cpx<T>);
    const size_t lds = (size_t)3 * tk * line;
    static bool init = false;
    if (!init) { allow_lds(k_fft_z_t<T, N2, TK>, (size_t)3 * TK * line); init = true; }
    const int64_t grid = ((int64_t)p->g.n1 * ntiles + E.nblk) * nrhs;
    k_fft_z_t<T, N2, TK><<<(unsigned)grid, 512, lds, s>>>(A, tb.tws[2], tb.half[0], tb.half[1], tb.half[2], spec,
                                                        sz, sy, nrhs, E);
}
template <typename T, int N2>
static void zpass(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s, const Tables<T> &tb, cpx<T> *spec,
                  int64_t sz, int64_t sy, const EnrUpd<T> &E) {
    if (p->fft_ztile[sizeof(T) == 8 ? 1 : 0])
        zpass_tk<T, N2, tkz_alt<T>(N2)>(p, A, nrhs, s, tb, spec, sz, sy, E);
    else
        zpass_tk<T, N2, tkz_t<T>(N2)>(p, A, nrhs, s, tb, spec, sz, sy, E);
}

// compile-time x and y passes (ztmpl sizes); return false when n has no such variant
template <typename T, int N> static void xfwd_t(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s,
                                                const cpx<T> *tw, T *f, const T *z, cpx<T> *spec) {
    const size_t lds = (size_t)XCfg<N>::PP * XCfg<N>::LS * sizeof(cpx<T>);
    static bool init = false;
    if (!init) { allow_lds(k_fft_x_fwd_t<T, N>, lds); init = true; }
    const int64_t npairs = (int64_t)3 * p->g.n2 * p->g.n1 / 2;
    const int64_t nblk = (npairs + XCfg<N>::PP - 1) / XCfg<N>::PP;
    k_fft_x_fwd_t<T, N><<<(unsigned)(nblk * nrhs), 256, lds, s>>>(A, tw, f, z, spec, nrhs);
}
template <typename T, int N> static void xinv_t(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s,
                                                const cpx<T> *tw, const cpx<T> *spec, int mode, T *out, T *u,
                                                T *d) {
    const size_t lds = (size_t)XCfg<N>::PP * XCfg<N>::LS * sizeof(cpx<T>);
    static bool init = false;
    if (!init) { allow_lds(k_fft_x_inv_t<T, N>, lds); init = true; }
    const int64_t npairs = (int64_t)3 * p->g.n2 * p->g.n1 / 2;
    const int64_t nblk = (npairs + XCfg<N>::PP - 1) / XCfg<N>::PP;
    k_fft_x_inv_t<T, N><<<(unsigned)(nblk * nrhs), 256, lds, s>>>(A, tw, spec, mode, out, u, d, nrhs);
}
template <typename T, int N1, bool INV> static void ypass_t(const xfft_problem *p, FftArgs A, int nrhs,
                                                           hipStream_t s, const cpx<T> *tw, cpx<T> *spec) {
    constexpr int TK = N1 >= 256 ? 8 : 16;
    const size_t lds = (size_t)TK * fft_ls(N1) * sizeof(cpx<T>);
    static bool init = false;
    if (!init) { allow_lds(k_fft_y_t<T, N1, TK, INV>, lds); init = true; }
    const int ntiles = (p->g.nh + TK - 1) / TK;
    const int64_t nblk = (int64_t)3 * p->g.n2 * ntiles;
    k_fft_y_t<T, N1, TK, INV><<<(unsigned)(nblk * nrhs), 256, lds, s>>>(A, tw, spec, nrhs);
}
template <typename T> static bool x_forward_t(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s,
                                              const cpx<T> *tw, T *f, const T *z, cpx<T> *spec) {
    switch (p->g.n0) {
        case 16: xfwd_t<T, 16>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 32: xfwd_t<T, 32>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 48: xfwd_t<T, 48>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 64: xfwd_t<T, 64>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 96: xfwd_t<T, 96>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 128: xfwd_t<T, 128>(p, A, nrhs, s, tw, f, z, spec); return true;
        case 256: xfwd_t<T, 256>(p, A, nrhs, s, tw, f, z, spec); return true;
        default: return false;
    }
}
template <typename T> static bool x_inverse_t(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s,
                                              const cpx<T> *tw, const cpx<T> *spec, int mode, T *out, T *u, T *d) {
    switch (p->g.n0) {
        case 16: xinv_t<T, 16>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 32: xinv_t<T, 32>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 48: xinv_t<T, 48>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 64: xinv_t<T, 64>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 96: xinv_t<T, 96>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 128: xinv_t<T, 128>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        case 256: xinv_t<T, 256>(p, A, nrhs, s, tw, spec, mode, out, u, d); return true;
        default: return false;
    }
}
template <typename T, bool INV> static bool y_pass_t(const xfft_problem *p, FftArgs A, int nrhs, hipStream_t s,
                                                     const cpx<T> *tw, cpx<T> *spec) {
    switch (p->g.n1) {
        case 16: ypass_t<T, 16, INV>(p, A, nrhs, s, tw, spec); return true;
        case 32: ypass_t<T, 32, INV>(p, A, nrhs, s, tw, spec); return true;
        case 48: ypass_t<T, 48, INV>(p, A, nrhs, s, tw, spec); return true;
        case 64: ypass_t<T, 64, INV>(p, A, nrhs, s, tw, spec); return true;
        case 96: ypass_t<T, 96, INV>(p, A, nrhs, s, tw, spec); return true;
        case 128: ypass_t<T, 128, INV>(p, A, nrhs, s, tw, spec); return true;
        case 256: ypass_t<T, 256, INV>(p, A, nrhs, s, tw, spec); return true;
        default: return false;
    }
}

template <typename T>
void launch_green_forward(xfft_problem *p, Work<T> &w, const Tables<T> &tb, T *f, const T *z, int nrhs,
                          const Flags *flags, int parity, hipStream_t s, int enr_mode, T *enr_out) {
    const Geometry &g = p->g;
    EnrUpd<T> E = enr_update_args<T>(p, w, enr_mode, enr_out);
    if (g.nX == 0) E.nblk = 0;
    FftArgs A = fft_args<T>(p, flags, parity);
    set_spec_layout<T>(p, A);
    const bool plane = use_plane<T>(p);
    int64_t sz, sy;
    if (plane) {
        sz = g.nh;
        sy = (int64_t)g.n2 * g.nh;
        xfft_prof_mark(p, -1, s);
        switch (g.n0) {
            case 16: plane_fwd<T, 16>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
            case 32: plane_fwd<T, 32>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
            case 48: plane_fwd<T, 48>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
            case 64: plane_fwd<T, 64>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
            case 96: plane_fwd<T, 96>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
            default: plane_fwd<T, 128>(p, A, nrhs, s, tb.tws[0], f, z, w.spec); break;
        }
        xfft_prof_mark(p, K_FFT_X_FWD + (sizeof(T) == 8 ? K_COUNT : 0), s);
    } else {
        sz = (int64_t)g.n1 * A.nhs;
        sy = A.nhs;
        {
            const int pp = pairs_for<T>(g.n0);
            const int64_t npairs = (int64_t)3 * g.n2 * g.n1 / 2;
            dim3 grid((unsigned)((npairs + pp - 1) / pp), nrhs);
            const size_t lds = (size_t)pp * (g.n0 + 1) * sizeof(cpx<T>);
            xfft_prof_mark(p, -1, s);
            if (!x_forward_t<T>(p, A, nrhs, s, tb.tws[0], f, z, w.spec))
                k_fft_x_fwd<T><<<grid, 256, lds, s>>>(A, p->plan[0], tb.tw[0], f, z, w.spec, pp);
            xfft_prof_mark(p, K_FFT_X_FWD + (sizeof(T) == 8 ? K_COUNT : 0), s);
        }
        {
            const int tk = tk_for<T>(g.n1, 1, 256);
            dim3 grid(3 * g.n2 * ((g.nh + tk - 1) / tk), nrhs);
            const size_t lds = (size_t)tk * (g.n1 + 1) * sizeof(cpx<T>);
            xfft_prof_mark(p, -1, s);
            if (!y_pass_t<T, false>(p, A, nrhs, s, tb.tws[1], w.spec))
                k_fft_y<T, false><<<grid, 256, lds, s>>>(A, p->plan[1], tb.tw[1], w.spec, tk);
            xfft_prof_mark(p, K_FFT_Y_FWD + (sizeof(T) == 8 ? K_COUNT : 0), s);
        }
    }
    {
        A.slot0 = p->slots.grn0;
        dim3 grid((unsigned)green_blocks<T>(p) * nrhs, 1);
        xfft_prof_mark(p, -1, s);
        if (ztmpl_size(g.n2)) {
            switch (g.n2) {
                case 16: zpass<T, 16>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                case 32: zpass<T, 32>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                case 48: zpass<T, 48>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                case 64: zpass<T, 64>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                case 96: zpass<T, 96>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                case 128: zpass<T, 128>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
                default: zpass<T, 256>(p, A, nrhs, s, tb, w.spec, sz, sy, E); break;
            }
        } else {
            const int tk = tk_z(g);
            const size_t lds = (size_t)3 * tk * (g.n2 + 1) * sizeof(cpx<T>);
            k_fft_z_green<T><<<grid, 512, lds, s>>>(A, p->plan[2], tb.tw[2], tb.half[0], tb.half[1], tb.half[2],
                                                     w.spec, tk, sz, sy);
        }
        xfft_prof_mark(p, K_FFT_Z_GREEN + (sizeof(T) == 8 ? K_COUNT : 0), s);
        // the generic z pass has no enriched workgroups
        if (!ztmpl_size(g.n2) && E.nblk) launch_enr_update<T>(p, w, enr_mode, enr_out, nrhs, flags, parity, s);
    }
    if (!plane) {
        const int tk = tk_for<T>(g.n1, 1, 256);
        dim3 grid(3 * g.n2 * ((g.nh + tk - 1) / tk), nrhs);
        const size_t lds = (size_t)tk * (g.n1 + 1) * sizeof(cpx<T>);
        xfft_prof_mark(p, -1, s);
        if (!y_pass_t<T, true>(p, A, nrhs, s, tb.tws[1], w.spec))
            k_fft_y<T, true><<<grid, 256, lds, s>>>(A, p->plan[1], tb.tw[1], w.spec, tk);
        xfft_prof_mark(p, K_FFT_Y_INV + (sizeof(T) == 8 ? K_COUNT : 0), s);
    }
}

template <typename T>
void launch_green_inverse(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int mode, T *out, int nrhs,
                          const Flags *flags, int parity, hipStream_t s, int enr_mode) {
    const Geometry &g = p->g;
    FftArgs A = fft_args<T>(p, flags, parity);
    set_spec_layout<T>(p, A);
    EnrFin<T> E = enr_final_args<T>(p, w, g.nX ? enr_mode : 0);
    xfft_prof_mark(p, -1, s);
    if (use_plane<T>(p)) {
        switch (g.n0) {
            case 16: plane_inv<T, 16>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
            case 32: plane_inv<T, 32>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
            case 48: plane_inv<T, 48>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
            case 64: plane_inv<T, 64>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
            case 96: plane_inv<T, 96>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
            default: plane_inv<T, 128>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d, E); break;
        }
        E.mode = 0;
    } else {
        const int pp = pairs_for<T>(g.n0);
        const int64_t npairs = (int64_t)3 * g.n2 * g.n1 / 2;
        dim3 grid((unsigned)((npairs + pp - 1) / pp), nrhs);
        const size_t lds = (size_t)pp * (g.n0 + 1) * sizeof(cpx<T>);
        if (!x_inverse_t<T>(p, A, nrhs, s, tb.tws[0], w.spec, mode, out, w.u, w.d))
            k_fft_x_inv<T><<<grid, 256, lds, s>>>(A, p->plan[0], tb.tw[0], w.spec, mode, out, w.u, w.d, pp);
    }
    xfft_prof_mark(p, K_FFT_X_INV + (sizeof(T) == 8 ? K_COUNT : 0), s);
    if (E.mode) launch_enr_final<T>(p, w, E.mode, nrhs, flags, parity, s);
}

template void launch_green_forward<double>(xfft_problem *, Work<double> &, const Tables<double> &, double *,
                                           const double *, int, const Flags *, int, hipStream_t, int, double *);
template void launch_green_forward<float>(xfft_problem *, Work<float> &, const Tables<float> &, float *,
                                          const float *, int, const Flags *, int, hipStream_t, int, float *);
template void launch_green_inverse<double>(xfft_problem *, Work<double> &, const Tables<double> &, int, double *,
                                           int, const Flags *, int, hipStream_t, int);
template void launch_green_inverse<float>(xfft_problem *, Work<float> &, const Tables<float> &, int, float *, int,
                                          const Flags *, int, hipStream_t, int);

}  // namespace xfft
