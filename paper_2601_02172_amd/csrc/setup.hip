// Setup of a problem on the device (Sec. 2, Sec. 3):
//  1. snap: L/h in voxel units, |L| < snap_eps -> 0 (Sec. 3); input validation;
//  2. classify every voxel: an element is cut when it has vertices with L > 0
//     and with L < 0; a voxel is irregular when it holds a cut element or
//     elements of different materials; vertices of cut elements are marked as
//     enriched nodes (eq. X-FEM space);
//  3. ordered compaction (block counts, one-block scan, in-order emit) of the
//     irregular voxels and of the enriched nodes (numbered by node index);
//  4. per irregular voxel: enriched index and level set of its corners and the
//     labels of its elements (decided once, in FP64);
//  5. D0_jj = sum over the cut elements at j of int ||M (grad N_X^j (x) I3)||^2
//     (eq. scaling factors) = 2 sum int |grad N_X^j|^2, gathered per enriched
//     node from its eight voxels through the per-side moments (element.h);
//  6. FFT twiddles exp(-2 pi i t / n) and half-angle tables sin, cos(pi k / n).
#include "kernels.h"
#include "element.h"
#include "fft_lines.h"

#include <cmath>
#include <vector>

namespace xfft {

namespace {

constexpr int SCAN_T = 256, SCAN_PER = 16, SCAN_CH = SCAN_T * SCAN_PER;

__device__ __forceinline__ int wrapn(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int64_t corner_node(int i, int j, int k, int c, int n0, int n1, int n2) {
    return wrapn(i + (c & 1), n0) + (int64_t)n0 * (wrapn(j + ((c >> 1) & 1), n1) + (int64_t)n1 * wrapn(k + (c >> 2), n2));
}

__global__ void k_snap(int64_t N, const double *L, double inv_h, double eps, const int32_t *phase, int nphase,
                       double *Ls, int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double v = L[i] * inv_h;
    if (!isfinite(v)) atomicOr(err, 1);
    const int ph = phase[i];
    if (ph < 0 || ph >= nphase) atomicOr(err, 2);
    Ls[i] = fabs(v) < eps ? 0.0 : v;
}

template <int t>
__device__ __forceinline__ void classify_tet(const double (&Lc)[8], const int (&pc)[8], bool &cut, int &lab_uncut,
                                             int &lp, int &ln, bool &ml) {
    double L[4];
    int lab[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { L[a] = Lc[tet_corner(t, a)]; lab[a] = pc[tet_corner(t, a)]; }
    const bool anyp = L[0] > 0 || L[1] > 0 || L[2] > 0 || L[3] > 0;
    const bool anyn = L[0] < 0 || L[1] < 0 || L[2] < 0 || L[3] < 0;
    cut = anyp && anyn;
    element_labels<double>(L, lab, lab_uncut, lp, ln, ml);
}

__global__ void k_classify(int n0, int n1, int n2, const double *Ls, const int32_t *phase, int p1, uint8_t *vflag,
                           int32_t *vlab, uint8_t *jflag, unsigned long long *counts) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int i = (int)(v % n0), j = (int)((v / n0) % n1), k = (int)(v / ((int64_t)n0 * n1));
    double Lc[8];
    int pc[8];
    int64_t nodes[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        nodes[c] = corner_node(i, j, k, c, n0, n1, n2);
        Lc[c] = Ls[nodes[c]];
        pc[c] = phase[nodes[c]];
    }
    if (p1) {
        // voxel-segmented P1: the level set at the voxel centre (mean of the
        // corners) picks the side; the corner with the largest |L| on that side
        // gives the material (first in corner order on ties)
        double sum = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) sum += Lc[c];
        const bool pos = sum >= 0.0;
        double best = -1.0;
        int lab = pc[0];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const bool on = pos ? Lc[c] >= 0.0 : Lc[c] < 0.0;
            if (on && fabs(Lc[c]) > best) { best = fabs(Lc[c]); lab = pc[c]; }
        }
        vflag[v] = 0;
        vlab[v] = lab;
        return;
    }
    bool cut[6], ml[6];
    int lu[6], lp[6], ln[6];
    classify_tet<0>(Lc, pc, cut[0], lu[0], lp[0], ln[0], ml[0]);
    classify_tet<1>(Lc, pc, cut[1], lu[1], lp[1], ln[1], ml[1]);
    classify_tet<2>(Lc, pc, cut[2], lu[2], lp[2], ln[2], ml[2]);
    classify_tet<3>(Lc, pc, cut[3], lu[3], lp[3], ln[3], ml[3]);
    classify_tet<4>(Lc, pc, cut[4], lu[4], lp[4], ln[4], ml[4]);
    classify_tet<5>(Lc, pc, cut[5], lu[5], lp[5], ln[5], ml[5]);
    bool irregular = false;
    int ncut = 0, nml = 0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        if (cut[t]) { irregular = true; ++ncut; nml += ml[t] ? 1 : 0; }
        if (lu[t] != lu[0]) irregular = true;
    }
    vflag[v] = irregular ? 1 : 0;
    vlab[v] = lu[0];
    if (ncut) {
        // vertices of cut elements are enriched (plain stores of the same value)
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            if (cut[t]) {
#pragma unroll
                for (int a = 0; a < 4; ++a) jflag[nodes[tet_corner(t, a)]] = 1;
            }
        }
        atomicAdd(&counts[0], (unsigned long long)ncut);
        if (nml) atomicAdd(&counts[1], (unsigned long long)nml);
    }
}

__global__ __launch_bounds__(SCAN_T) void k_scan_count(int64_t n, const uint8_t *flag, int32_t *cnt) {
    __shared__ double red[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CH;
    double c[1] = {0.0};
    for (int q = 0; q < SCAN_PER; ++q) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_PER + q;
        if (i < n && flag[i]) c[0] += 1.0;
    }
    block_sum<1>(c, red);
    if (threadIdx.x == 0) cnt[blockIdx.x] = (int32_t)c[0];
}

__global__ __launch_bounds__(1024) void k_scan_offsets(int nb, const int32_t *cnt, int32_t *off, int64_t *total) {
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const int64_t v = (i < nb) ? cnt[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t add = (threadIdx.x >= o) ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) off[i] = (int32_t)(carry + buf[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Emit in order: for voxels, irr[pos] = v and vmat[v] = -(pos + 1) (or the label);
// for nodes, jlist[pos] = node and jmap[node] = pos (or -1).
__global__ __launch_bounds__(SCAN_T) void k_scan_emit(int64_t n, const uint8_t *flag, const int32_t *off,
                                                       int32_t *list, int32_t *map, const int32_t *lab) {
    __shared__ int32_t pre[SCAN_T];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CH + (int64_t)threadIdx.x * SCAN_PER;
    int c = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        const int64_t i = base + q;
        if (i < n && flag[i]) ++c;
    }
    pre[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        const int add = (threadIdx.x >= o) ? pre[threadIdx.x - o] : 0;
        __syncthreads();
        pre[threadIdx.x] += add;
        __syncthreads();
    }
    int pos = off[blockIdx.x] + pre[threadIdx.x] - c;
    for (int q = 0; q < SCAN_PER; ++q) {
        const int64_t i = base + q;
        if (i >= n) break;
        if (flag[i]) {
            list[pos] = (int32_t)i;
            map[i] = lab ? -(pos + 1) : pos;
            ++pos;
        } else {
            map[i] = lab ? lab[i] : -1;
        }
    }
}

template <int t>
__device__ __forceinline__ void irr_labels_tet(const double (&Lc)[8], const int (&pc)[8], int32_t *out,
                                               int64_t stride) {
    bool cut, ml;
    int lu, lp, ln;
    classify_tet<t>(Lc, pc, cut, lu, lp, ln, ml);
    out[(2 * t) * stride] = cut ? lp : lu;
    out[(2 * t + 1) * stride] = cut ? ln : lu;
}

__global__ void k_irr_tables(int64_t nirr, int n0, int n1, int n2, const int32_t *irr, const double *Ls,
                             const int32_t *phase, const int32_t *jmap, int32_t *irr_j, int32_t *irr_lab,
                             double *irr_L64, float *irr_L32) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nirr) return;
    const int64_t v = irr[q];
    const int i = (int)(v % n0), j = (int)((v / n0) % n1), k = (int)(v / ((int64_t)n0 * n1));
    double Lc[8];
    int pc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t nd = corner_node(i, j, k, c, n0, n1, n2);
        Lc[c] = Ls[nd];
        pc[c] = phase[nd];
        irr_j[c * nirr + q] = jmap[nd];
        irr_L64[c * nirr + q] = Lc[c];
        irr_L32[c * nirr + q] = (float)Lc[c];
    }
    int32_t *lab = irr_lab + q;
    irr_labels_tet<0>(Lc, pc, lab, nirr);
    irr_labels_tet<1>(Lc, pc, lab, nirr);
    irr_labels_tet<2>(Lc, pc, lab, nirr);
    irr_labels_tet<3>(Lc, pc, lab, nirr);
    irr_labels_tet<4>(Lc, pc, lab, nirr);
    irr_labels_tet<5>(Lc, pc, lab, nirr);
}

// Side moments of the six Kuhn tets of every irregular voxel (exact
// integration over the two sides of a cut element): geometry only, so they are
// computed once per setup in FP64 instead of in every operator application.
// Stored per tet, 10 values [t][e][qv] (irregular voxel fastest, so that the
// lanes of a wave read consecutive words): the upper triangle (row by row) of
// the moments of the side with the smaller volume, whose entry 0 carries the
// sign bit when that side is the - side (all moments are >= 0).  The operator
// forms the other side as the complement M^tet - Ms, which is accurate in FP32
// because it is the larger side.
__global__ void k_irr_moments(int64_t nirr, const double *irr_L64, double *M64, float *M32) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nirr) return;
    double Lc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Lc[c] = irr_L64[c * nirr + q];
    for (int t = 0; t < 6; ++t) {
        double L[4];
        bool anyp = false, anyn = false;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            L[a] = Lc[tet_corner(t, a)];
            anyp |= L[a] > 0.0;
            anyn |= L[a] < 0.0;
        }
        double Ms[4][4];
        bool pos = true;
        if (anyp && anyn) {
            pos = small_side_moments<double>(L, 1.0 / 6.0, Ms);
            // keep the side of smaller volume (sum of the moments): its
            // complement is then the larger side and is formed accurately in FP32
            const double Vt = (1.0 / 6.0) * 0.05;
            double vs = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int d = 0; d < 4; ++d) vs += Ms[c][d];
            if (vs > 0.5 * (20.0 * Vt)) {      // the whole tet: sum of V (1 + delta_cd) / 20 = V
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int d = 0; d < 4; ++d) Ms[c][d] = Vt * (c == d ? 2.0 : 1.0) - Ms[c][d];
                pos = !pos;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int d = 0; d < 4; ++d) Ms[c][d] = 0.0;
        }
        double v[10];
        int k = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = c; d < 4; ++d, ++k) v[k] = Ms[c][d];
        if (!pos) v[0] = -v[0];                       // sign bit marks the - side (also for +0)
#pragma unroll
        for (int e = 0; e < 10; ++e) {
            M64[(t * 10 + e) * nirr + q] = v[e];
            M32[(t * 10 + e) * nirr + q] = (float)v[e];
        }
    }
}

// int over both sides of |grad N_X^a|^2 for vertex a of cut Kuhn tet t
template <int t>
__device__ __forceinline__ double d0_tet(const double (&Lc)[8], int corner) {
    double L[4];
    int a = -1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        L[v] = Lc[tet_corner(t, v)];
        if (tet_corner(t, v) == corner) a = v;
    }
    if (a < 0) return 0.0;
    const bool anyp = L[0] > 0 || L[1] > 0 || L[2] > 0 || L[3] > 0;
    const bool anyn = L[0] < 0 || L[1] < 0 || L[2] < 0 || L[3] < 0;
    if (!(anyp && anyn)) return 0.0;
    double Mp[4][4], Mm[4][4];
    side_moments<double>(L, 1.0 / 6.0, Mp, Mm);
    double ga[3];
    kuhn_g<t, double>(a, ga);
    const double g2 = ga[0] * ga[0] + ga[1] * ga[1] + ga[2] * ga[2];
    double tot = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? 1.0 : -1.0;
        double w[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) w[b] = fabs(L[b]) - sg * L[b];
        double G[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double gb[3];
            kuhn_g<t, double>(b, gb);
            G[0] += w[b] * gb[0]; G[1] += w[b] * gb[1]; G[2] += w[b] * gb[2];
        }
        // int |w_c g_a + delta_ac G|^2 weights: g2 w^T M w + 2 (g_a . G) (M w)_a + M_aa |G|^2
        double wMw = 0.0, Mwa = 0.0, Maa = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double rowc = 0.0;
#pragma unroll
            for (int d = 0; d < 4; ++d) rowc += (side == 0 ? Mp[c][d] : Mm[c][d]) * w[d];
            wMw += w[c] * rowc;
            if (c == a) { Mwa = rowc; Maa = side == 0 ? Mp[c][c] : Mm[c][c]; }
        }
        const double gG = ga[0] * G[0] + ga[1] * G[1] + ga[2] * G[2];
        const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        tot += g2 * wMw + 2.0 * gG * Mwa + Maa * G2;
    }
    return tot;
}

__global__ void k_d0(int64_t nX, int n0, int n1, int n2, const int32_t *jlist, const int32_t *vmat,
                     const double *irr_L64, int64_t nirr, double scale, double *d0, double *d0is64,
                     float *d0is32) {
    const int64_t jn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jn >= nX) return;
    const int64_t node = jlist[jn];
    const int i = (int)(node % n0), j = (int)((node / n0) % n1), k = (int)(node / ((int64_t)n0 * n1));
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int64_t vox = wrapn(i - (c & 1), n0) + (int64_t)n0 * (wrapn(j - ((c >> 1) & 1), n1) + (int64_t)n1 * wrapn(k - (c >> 2), n2));
        const int m = vmat[vox];
        if (m >= 0) continue;
        const int64_t q = -(int64_t)m - 1;
        double Lc[8];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) Lc[cc] = irr_L64[cc * nirr + q];
        acc += d0_tet<0>(Lc, c) + d0_tet<1>(Lc, c) + d0_tet<2>(Lc, c) + d0_tet<3>(Lc, c) + d0_tet<4>(Lc, c) +
               d0_tet<5>(Lc, c);
    }
    // eq. scaling factors with the norm of the scalar function's gradient:
    // D0_jj = int |grad N_X^j|^2 (the reading that gives the paper's iteration
    // counts for the Hashin inclusion, Sec. 4.2)
    const double D = acc * scale;
    d0[jn] = D;
    d0is64[jn] = 1.0 / sqrt(D);
    d0is32[jn] = (float)(1.0 / sqrt(D));
}

__global__ void k_enr_src(int64_t nX, int n0, int n1, int n2, const int32_t *jlist, const int32_t *vmat,
                          int32_t *src) {
    const int64_t jn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jn >= nX) return;
    const int64_t node = jlist[jn];
    const int i = (int)(node % n0), j = (int)((node / n0) % n1), k = (int)(node / ((int64_t)n0 * n1));
    for (int c = 0; c < 8; ++c) {
        const int64_t vox = wrapn(i - (c & 1), n0) + (int64_t)n0 * (wrapn(j - ((c >> 1) & 1), n1) + (int64_t)n1 * wrapn(k - (c >> 2), n2));
        const int m = vmat[vox];
        src[jn * 8 + c] = (m < 0) ? (int32_t)(8 * (-(int64_t)m - 1) + c) : -1;
    }
}

__global__ void k_fft_tables(int n, double2 *tw64, float2 *tw32, double *half64, float *half32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double s, c;
    sincospi(-2.0 * (double)t / (double)n, &s, &c);
    tw64[t] = make_double2(c, s);
    tw32[t] = make_float2((float)c, (float)s);
    double hs, hc;
    sincospi((double)t / (double)n, &hs, &hc);
    half64[2 * t] = hs;
    half64[2 * t + 1] = hc;
    half32[2 * t] = (float)hs;
    half32[2 * t + 1] = (float)hc;
}

// stage-major twiddle tables (gathered from the natural-order ones, so the
// values are identical)
__global__ void k_fft_stage_tables(int n, const double2 *tw64, const float2 *tw32, double2 *st64, float2 *st32) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int t = e < n - 1 ? fft_stage_index(n, e) : -1;
    st64[e] = t >= 0 ? tw64[t] : make_double2(1.0, 0.0);
    st32[e] = t >= 0 ? tw32[t] : make_float2(1.0f, 0.0f);
}

__global__ void k_lame(int n, const double *lame, float *lame32) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * n) lame32[t] = (float)lame[t];
}

#define CK(x)                                 \
    do {                                      \
        if ((x) != hipSuccess) return XFFT_EDEVICE_INTERNAL; \
    } while (0)

constexpr int XFFT_EDEVICE_INTERNAL = -3;
constexpr int XFFT_ENOMEM_INTERNAL = -2;
constexpr int XFFT_EINVAL_INTERNAL = -1;

int compact(hipStream_t s, int64_t n, const uint8_t *flag, int32_t *map, const int32_t *lab, int32_t **list_out,
            int64_t *count_out) {
    const int nb = (int)((n + SCAN_CH - 1) / SCAN_CH);
    int32_t *cnt = nullptr, *off = nullptr;
    int64_t *tot = nullptr;
    if (hipMalloc(&cnt, sizeof(int32_t) * nb) != hipSuccess) return XFFT_ENOMEM_INTERNAL;
    if (hipMalloc(&off, sizeof(int32_t) * nb) != hipSuccess) { (void)hipFree(cnt); return XFFT_ENOMEM_INTERNAL; }
    if (hipMalloc(&tot, sizeof(int64_t)) != hipSuccess) { (void)hipFree(cnt); (void)hipFree(off); return XFFT_ENOMEM_INTERNAL; }
    k_scan_count<<<nb, SCAN_T, 0, s>>>(n, flag, cnt);
    k_scan_offsets<<<1, 1024, 0, s>>>(nb, cnt, off, tot);
    int64_t total = 0;
    int rc = 0;
    if (hipMemcpyAsync(&total, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = XFFT_EDEVICE_INTERNAL;
    int32_t *list = nullptr;
    if (!rc && hipMalloc(&list, sizeof(int32_t) * (total > 0 ? total : 1)) != hipSuccess) rc = XFFT_ENOMEM_INTERNAL;
    if (!rc) k_scan_emit<<<nb, SCAN_T, 0, s>>>(n, flag, off, list, map, lab);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = XFFT_EDEVICE_INTERNAL;
    (void)hipFree(cnt);
    (void)hipFree(off);
    (void)hipFree(tot);
    if (rc) { if (list) (void)hipFree(list); return rc; }
    *list_out = list;
    *count_out = total;
    return 0;
}

}  // namespace

// L_dev_raw: device copy of the caller's level set (units of len).
int run_setup(xfft_problem *p, const double *L_dev_raw) {
    hipStream_t s = p->stream;
    Geometry &g = p->g;
    const int64_t N = g.N;
    const int tb = 256;
    const unsigned nbN = (unsigned)((N + tb - 1) / tb);
    int *err = nullptr;
    unsigned long long *counts = nullptr;
    uint8_t *vflag = nullptr, *jflag = nullptr;
    int32_t *vlab = nullptr, *jmap = nullptr;
    int rc = 0;
    auto cleanup = [&]() {
        if (err) (void)hipFree(err);
        if (counts) (void)hipFree(counts);
        if (vflag) (void)hipFree(vflag);
        if (jflag) (void)hipFree(jflag);
        if (vlab) (void)hipFree(vlab);
        if (jmap) (void)hipFree(jmap);
    };
    if (hipMalloc(&err, sizeof(int)) != hipSuccess || hipMalloc(&counts, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&vflag, N) != hipSuccess || hipMalloc(&jflag, N) != hipSuccess ||
        hipMalloc(&vlab, 4 * N) != hipSuccess || hipMalloc(&jmap, 4 * N) != hipSuccess) {
        cleanup();
        return XFFT_ENOMEM_INTERNAL;
    }
    if (hipMemsetAsync(err, 0, sizeof(int), s) != hipSuccess ||
        hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s) != hipSuccess ||
        hipMemsetAsync(jflag, 0, N, s) != hipSuccess) {
        cleanup();
        return XFFT_EDEVICE_INTERNAL;
    }
    k_snap<<<nbN, tb, 0, s>>>(N, L_dev_raw, 1.0 / p->h, p->snap_eps, p->phase, g.nphase, p->Ls, err);
    int herr = 0;
    if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return XFFT_EDEVICE_INTERNAL;
    }
    if (herr) {
        cleanup();
        return XFFT_EINVAL_INTERNAL;
    }
    k_classify<<<nbN, tb, 0, s>>>(g.n0, g.n1, g.n2, p->Ls, p->phase, p->p1, vflag, vlab, jflag, counts);
    rc = compact(s, N, vflag, p->vmat, vlab, &p->irr, &g.nirr);
    if (!rc) rc = compact(s, N, jflag, jmap, nullptr, &p->jlist, &g.nX);
    unsigned long long hc[2] = {0, 0};
    if (!rc && (hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
        rc = XFFT_EDEVICE_INTERNAL;
    p->n_cut_elements = (int64_t)hc[0];
    p->n_multilabel = (int64_t)hc[1];
    const int64_t nirr = g.nirr > 0 ? g.nirr : 1, nX = g.nX > 0 ? g.nX : 1;
    if (!rc) {
        if (hipMalloc(&p->irr_j, sizeof(int32_t) * 8 * nirr) != hipSuccess ||
            hipMalloc(&p->irr_lab, sizeof(int32_t) * 12 * nirr) != hipSuccess ||
            hipMalloc(&p->t64.irr_L, sizeof(double) * 8 * nirr) != hipSuccess ||
            hipMalloc(&p->t32.irr_L, sizeof(float) * 8 * nirr) != hipSuccess ||
            hipMalloc(&p->t64.irr_M, sizeof(double) * 60 * nirr) != hipSuccess ||
            hipMalloc(&p->t32.irr_M, sizeof(float) * 60 * nirr) != hipSuccess ||
            hipMalloc(&p->d0, sizeof(double) * nX) != hipSuccess ||
            hipMalloc(&p->t64.d0is, sizeof(double) * nX) != hipSuccess ||
            hipMalloc(&p->t32.d0is, sizeof(float) * nX) != hipSuccess ||
            hipMalloc(&p->enr_src, sizeof(int32_t) * 8 * nX) != hipSuccess)
            rc = XFFT_ENOMEM_INTERNAL;
    }
    if (!rc && g.nirr > 0) {
        k_irr_tables<<<(unsigned)((g.nirr + tb - 1) / tb), tb, 0, s>>>(g.nirr, g.n0, g.n1, g.n2, p->irr, p->Ls,
                                                                       p->phase, jmap, p->irr_j, p->irr_lab,
                                                                       p->t64.irr_L, p->t32.irr_L);
        k_irr_moments<<<(unsigned)((g.nirr + tb - 1) / tb), tb, 0, s>>>(g.nirr, p->t64.irr_L, p->t64.irr_M,
                                                                        p->t32.irr_M);
    }
    if (!rc && g.nX > 0) {
        k_d0<<<(unsigned)((g.nX + tb - 1) / tb), tb, 0, s>>>(g.nX, g.n0, g.n1, g.n2, p->jlist, p->vmat, p->t64.irr_L,
                                                             g.nirr, p->d0_scale, p->d0, p->t64.d0is, p->t32.d0is);
        k_enr_src<<<(unsigned)((g.nX + tb - 1) / tb), tb, 0, s>>>(g.nX, g.n0, g.n1, g.n2, p->jlist, p->vmat,
                                                                  p->enr_src);
    }
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = XFFT_EDEVICE_INTERNAL;
    if (!rc && hipGetLastError() != hipSuccess) rc = XFFT_EDEVICE_INTERNAL;
    cleanup();
    return rc;
}

int compute_tables(xfft_problem *p) {
    hipStream_t s = p->stream;
    const int n[3] = {p->g.n0, p->g.n1, p->g.n2};
    for (int a = 0; a < 3; ++a) {
        p->plan[a] = make_plan(n[a]);
        if (hipMalloc(&p->t64.tw[a], sizeof(cpx<double>) * n[a]) != hipSuccess ||
            hipMalloc(&p->t32.tw[a], sizeof(cpx<float>) * n[a]) != hipSuccess ||
            hipMalloc(&p->t64.half[a], sizeof(double) * 2 * n[a]) != hipSuccess ||
            hipMalloc(&p->t32.half[a], sizeof(float) * 2 * n[a]) != hipSuccess ||
            hipMalloc(&p->t64.tws[a], sizeof(cpx<double>) * n[a]) != hipSuccess ||
            hipMalloc(&p->t32.tws[a], sizeof(cpx<float>) * n[a]) != hipSuccess)
            return XFFT_ENOMEM_INTERNAL;
        k_fft_tables<<<(n[a] + 255) / 256, 256, 0, s>>>(n[a], reinterpret_cast<double2 *>(p->t64.tw[a]),
                                                        reinterpret_cast<float2 *>(p->t32.tw[a]), p->t64.half[a],
                                                        p->t32.half[a]);
        k_fft_stage_tables<<<(n[a] + 255) / 256, 256, 0, s>>>(
            n[a], reinterpret_cast<const double2 *>(p->t64.tw[a]), reinterpret_cast<const float2 *>(p->t32.tw[a]),
            reinterpret_cast<double2 *>(p->t64.tws[a]), reinterpret_cast<float2 *>(p->t32.tws[a]));
    }
    const int np = p->g.nphase;
    if (hipMalloc(&p->t64.lame, sizeof(double) * 2 * np) != hipSuccess ||
        hipMalloc(&p->t32.lame, sizeof(float) * 2 * np) != hipSuccess)
        return XFFT_ENOMEM_INTERNAL;
    if (hipMemcpyAsync(p->t64.lame, p->lame_host.data(), sizeof(double) * 2 * np, hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return XFFT_EDEVICE_INTERNAL;
    k_lame<<<(2 * np + 255) / 256, 256, 0, s>>>(np, p->t64.lame, p->t32.lame);
    if (hipStreamSynchronize(s) != hipSuccess) return XFFT_EDEVICE_INTERNAL;
    return 0;
}

}  // namespace xfft
