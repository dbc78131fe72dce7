// CG recurrences of Algorithm 1 on the device (FP64 scalars for every
// precision), the enriched-block vector updates (the preconditioner is the
// identity on the scaled enriched dofs, eq. scaledPreconditioner) and the
// helpers of iterative refinement.
//
// Stopping criteria (eq. stoppingCriterion, residual of eq. convergence
// normalised by |Y|): crit 0: sqrt(res2 / |Y|) <= tol ||<sigma>||; crit 1
// (inner solves of iterative refinement): res2 <= tol_inner^2 res2_0, or the
// criterion-0 test with tol scaled by INNER_MARGIN.  In an inner solve sigma
// holds the average stress of the outer iterate (the correction's stress is not
// tracked), so the second test ends the last inner solve as soon as its
// recursive residual meets the outer tolerance, instead of after a full
// tol_inner reduction.
#include "xfft.h"
#include "kernels.h"
#include "enriched.h"

namespace xfft {

namespace {

// share of the outer tolerance an inner solve aims for: the FP64 residual of
// the corrected iterate differs from the inner recursive residual by FP32
// rounding of the correction, far below this margin
constexpr double INNER_MARGIN = 0.5;

struct ScArgs {
    const double *partial;
    int nslots;
    int s0, n;            // slot range to sum
    int s1, n1;           // second slot range (0 length when unused)
    Scalars *scal;
    Flags *flags;
    double volume;
    int op, crit, parity, maxit;
    int scheme;           // XFFT_LCG, XFFT_NLCG, XFFT_BB or XFFT_BASIC
    double *sum_out;      // [rhs][7] or null
};

__global__ __launch_bounds__(256) void k_scalars(ScArgs A) {
    __shared__ double red[4 * 7];
    const int r = blockIdx.x;
    Flags &F = A.flags[r];
    const bool act = (A.op == SC_ALPHA || A.op == SC_BETA) ? F.active[A.parity] != 0 : true;
    if (!act) {
        // an inactive right-hand side stays inactive in the next iteration too
        if (A.op == SC_BETA && threadIdx.x == 0) F.active[1 - A.parity] = 0;
        return;
    }
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    const double *P = A.partial + ((int64_t)r * A.nslots + A.s0) * NPART;
    for (int i = threadIdx.x; i < A.n; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] += P[(int64_t)i * NPART + q];
    }
    const double *P1 = A.partial + ((int64_t)r * A.nslots + A.s1) * NPART;
    for (int i = threadIdx.x; i < A.n1; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] += P1[(int64_t)i * NPART + q];
    }
    block_sum<7>(v, red);
    if (threadIdx.x != 0) return;
    Scalars &S = A.scal[r];
    if (A.sum_out) {
#pragma unroll
        for (int q = 0; q < 7; ++q) A.sum_out[r * 7 + q] = v[q];
    }
    const double r2 = 1.41421356237309504880;
    if (A.op == SC_INIT_SIGMA) {
        // Mandel average stress from the stress integral (tensor components)
        S.sigma[0] = v[1] / A.volume; S.sigma[1] = v[2] / A.volume; S.sigma[2] = v[3] / A.volume;
        S.sigma[3] = r2 * v[4] / A.volume; S.sigma[4] = r2 * v[5] / A.volume; S.sigma[5] = r2 * v[6] / A.volume;
        S.alpha = 0.0;
        S.beta = 0.0;
    } else if (A.op == SC_INIT_RES) {
        S.res2 = v[0];
        S.res2_0 = v[0];
        double sn = 0.0;
        for (int q = 0; q < 6; ++q) sn += S.sigma[q] * S.sigma[q];
        const double res = sqrt(fmax(v[0], 0.0) / A.volume);
        const bool conv = (A.crit == 0) ? (res <= S.tol * sqrt(sn)) : (v[0] <= 0.0);
        F.conv = conv ? 1 : 0;
        F.pad[0] = conv ? 1 : 0;
        F.breakdown = 0;
        F.active[0] = (!conv && A.maxit > F.iters && isfinite(v[0])) ? 1 : 0;
        F.active[1] = 0;
    } else if (A.op == SC_ALPHA) {
        const double zd = v[0];
        if (!(zd > 0.0) || !isfinite(zd)) {
            F.breakdown = 1;
            S.alpha = 0.0;
            return;
        }
        // step of the scheme (Sec. 3, solvers): linear CG takes the exact line
        // search, the basic scheme and nonlinear CG the fixed step s0, and
        // Barzilai-Borwein the line-search step of the previous iteration
        double alpha = S.res2 / zd;
        if (A.scheme == XFFT_NLCG || A.scheme == XFFT_BASIC) {
            alpha = S.s0;
        } else if (A.scheme == XFFT_BB) {
            alpha = S.alpha_lag > 0.0 ? S.alpha_lag : S.s0;
            S.alpha_lag = S.res2 / zd;
        }
        S.alpha = alpha;
        S.sigma[0] += alpha * v[1] / A.volume; S.sigma[1] += alpha * v[2] / A.volume;
        S.sigma[2] += alpha * v[3] / A.volume;
        S.sigma[3] += alpha * r2 * v[4] / A.volume; S.sigma[4] += alpha * r2 * v[5] / A.volume;
        S.sigma[5] += alpha * r2 * v[6] / A.volume;
    } else if (A.op == SC_BETA) {
        const double rn = v[0];
        // the basic and Barzilai-Borwein schemes step along y = P^-1 f
        const bool cg = A.scheme == XFFT_LCG || A.scheme == XFFT_NLCG;
        S.beta = (cg && S.res2 > 0.0) ? rn / S.res2 : 0.0;
        S.res2 = rn;
        F.iters += 1;
        double sn = 0.0;
        for (int q = 0; q < 6; ++q) sn += S.sigma[q] * S.sigma[q];
        const double res = sqrt(fmax(rn, 0.0) / A.volume);
        const double target = S.tol * sqrt(sn);
        bool conv = (A.crit == 0) ? (res <= target)
                                  : (rn <= S.tol_inner * S.tol_inner * S.res2_0 || res <= INNER_MARGIN * target);
        if (!isfinite(rn)) F.breakdown = 1;
        F.conv = conv ? 1 : 0;
        F.active[1 - A.parity] = (!conv && !F.breakdown && F.iters < A.maxit) ? 1 : 0;
    }
}

template <typename T>
__global__ __launch_bounds__(ENR_BLOCK) void k_enr_update(EnrUpd<T> E, const Flags *flags, int parity,
                                                           const Scalars *scal, double *partial, int nslots) {
    __shared__ double red[ENR_BLOCK / 64];
    const int r = blockIdx.y;
    if (flags && !flags[r].active[parity]) return;
    enr_update_block<T>(E, scal, partial, nslots, r, blockIdx.x, red);
}

template <typename T>
__global__ __launch_bounds__(256) void k_enr_final(EnrFin<T> E, const Flags *flags, int parity, const Scalars *scal) {
    const int r = blockIdx.y;
    if (flags && !flags[r].active[parity]) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    enr_final_rows<T>(E, scal, r, j, E.nX);
}

// iterative refinement: w32.f <- (float) w64.f, w32.u <- 0 for RHS whose outer loop runs
__global__ void k_round(int64_t n, const Flags *flags, const double *src, float *dst, float *zero_dst) {
    const int r = blockIdx.y;
    if (flags && flags[r].pad[0] != 0) return;      // pad[0]: outer loop finished
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[(int64_t)r * n + i] = (float)src[(int64_t)r * n + i];
    zero_dst[(int64_t)r * n + i] = 0.0f;
}

__global__ void k_accumulate(int64_t n, const Flags *flags, double *dst, const float *src) {
    const int r = blockIdx.y;
    if (flags && flags[r].pad[0] != 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[(int64_t)r * n + i] += (double)src[(int64_t)r * n + i];
}

}  // namespace

void launch_scalars(xfft_problem *p, int op, int crit, int nrhs, int parity, double *sum_out, hipStream_t s,
                    bool fp64) {
    ScArgs A;
    A.partial = p->partial;
    A.nslots = p->nslots;
    const SlotLayout &L = p->slots;
    if (op == SC_INIT_SIGMA || op == SC_ALPHA || op == SC_SUM_ONLY) {
        A.s0 = L.fe0;
        A.n = L.fe_n;
        // irregular-voxel slots of the kernel the last operator launch used
        // (moment form: before the enriched ones; cached matrices: after them)
        A.s1 = p->last_op_vm ? L.enr0 : L.cut0;
        A.n1 = p->last_op_vm ? L.enr_n + L.vm_n : L.cut_n + L.enr_n;
    } else {
        A.s0 = L.grn0;
        A.n = fp64 ? green_blocks<double>(p) : green_blocks<float>(p);
        A.s1 = L.eu0;
        A.n1 = L.eu_n;
    }
    A.scal = p->scal;
    A.flags = p->flags;
    A.volume = (double)p->g.N;
    A.op = op;
    A.crit = crit;
    A.parity = parity;
    A.maxit = p->maxit;
    A.scheme = p->scheme;
    A.sum_out = sum_out;
    xfft_prof_mark(p, -1, s);
    k_scalars<<<nrhs, 256, 0, s>>>(A);
    xfft_prof_mark(p, K_SCALARS + K_COUNT, s);
}

template <typename T>
EnrUpd<T> enr_update_args(xfft_problem *p, Work<T> &w, int mode, T *out) {
    EnrUpd<T> E;
    E.nX = p->g.nX;
    E.mode = mode;
    E.fe = w.fe;
    E.ze = w.ze;
    E.out = out;
    E.nblk = p->slots.eu_n;
    E.slot0 = p->slots.eu0;
    return E;
}

template <typename T>
EnrFin<T> enr_final_args(xfft_problem *p, Work<T> &w, int mode) {
    EnrFin<T> E;
    E.nX = p->g.nX;
    E.mode = mode;
    E.ue = w.ue;
    E.de = w.de;
    E.fe = w.fe;
    return E;
}

template <typename T>
void launch_enr_update(xfft_problem *p, Work<T> &w, int mode, T *out, int nrhs, const Flags *flags, int parity,
                       hipStream_t s) {
    if (p->g.nX == 0) return;
    dim3 grid(p->slots.eu_n, nrhs);
    xfft_prof_mark(p, -1, s);
    k_enr_update<T><<<grid, ENR_BLOCK, 0, s>>>(enr_update_args<T>(p, w, mode, out), flags, parity, p->scal,
                                               p->partial, p->nslots);
    xfft_prof_mark(p, K_ENR_UPDATE + (sizeof(T) == 8 ? K_COUNT : 0), s);
}

template <typename T>
void launch_enr_final(xfft_problem *p, Work<T> &w, int mode, int nrhs, const Flags *flags, int parity,
                      hipStream_t s) {
    if (p->g.nX == 0) return;
    dim3 grid((unsigned)((p->g.nX + 255) / 256), nrhs);
    xfft_prof_mark(p, -1, s);
    k_enr_final<T><<<grid, 256, 0, s>>>(enr_final_args<T>(p, w, mode), flags, parity, p->scal);
    xfft_prof_mark(p, K_ENR_FINAL + (sizeof(T) == 8 ? K_COUNT : 0), s);
}

template EnrUpd<double> enr_update_args<double>(xfft_problem *, Work<double> &, int, double *);
template EnrUpd<float> enr_update_args<float>(xfft_problem *, Work<float> &, int, float *);
template EnrFin<double> enr_final_args<double>(xfft_problem *, Work<double> &, int);
template EnrFin<float> enr_final_args<float>(xfft_problem *, Work<float> &, int);
template void launch_enr_update<double>(xfft_problem *, Work<double> &, int, double *, int, const Flags *, int,
                                        hipStream_t);
template void launch_enr_update<float>(xfft_problem *, Work<float> &, int, float *, int, const Flags *, int,
                                       hipStream_t);
template void launch_enr_final<double>(xfft_problem *, Work<double> &, int, int, const Flags *, int, hipStream_t);
template void launch_enr_final<float>(xfft_problem *, Work<float> &, int, int, const Flags *, int, hipStream_t);

void launch_round_to_float(xfft_problem *p, int nrhs, hipStream_t s) {
    const int64_t nf = 3 * p->g.N, ne = 3 * p->g.nX;
    k_round<<<dim3((unsigned)((nf + 255) / 256), nrhs), 256, 0, s>>>(nf, p->flags, p->w64.f, p->w32.f, p->w32.u);
    if (ne > 0)
        k_round<<<dim3((unsigned)((ne + 255) / 256), nrhs), 256, 0, s>>>(ne, p->flags, p->w64.fe, p->w32.fe,
                                                                         p->w32.ue);
}

void launch_accumulate_correction(xfft_problem *p, int nrhs, hipStream_t s) {
    const int64_t nf = 3 * p->g.N, ne = 3 * p->g.nX;
    k_accumulate<<<dim3((unsigned)((nf + 255) / 256), nrhs), 256, 0, s>>>(nf, p->flags, p->w64.u, p->w32.u);
    if (ne > 0)
        k_accumulate<<<dim3((unsigned)((ne + 255) / 256), nrhs), 256, 0, s>>>(ne, p->flags, p->w64.ue, p->w32.ue);
}

}  // namespace xfft
