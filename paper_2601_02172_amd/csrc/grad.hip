// Lame-parameter derivative of the energy form of C_eff (App. A, Galerkin
// orthogonality): with eps_k = eps_bar_k + grad^s u_k for the six unit Mandel
// loads,
//   dC_kl / dlambda_p = |Y|^-1 int_p tr eps_k tr eps_l,
//   dC_kl / dmu_p     = 2 |Y|^-1 int_p eps_k : eps_l.
// Regular voxels: constant strain per element.  Cut elements: on each side the
// strain is linear, eps(x) = sum_c lambda_c(x) eps_c, so int eps_k : eps_l =
// sum_cd M_cd eps_kc : eps_ld with the side's second-moment matrix M; writing
// M = R R^T (Cholesky) turns this into four weighted "virtual points"
// eps~_k,j = sum_c R_cj eps_kc with unit weights.
// Per-phase sums: each block accumulates a [nphase][42] table in LDS (21 pairs
// k <= l for lambda, 21 for mu) and writes it out; a second kernel sums the
// block tables in a fixed order.
#include "kernels.h"
#include "element.h"

namespace xfft {

namespace {

constexpr int NPAIR = 21;
constexpr int NG = 2 * NPAIR;
constexpr int GT = 256;

__device__ __forceinline__ int wrapg(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// accumulate products of six strains (tensor components) with weight wgt into acc[42]
__device__ __forceinline__ void add_products(double (&acc)[NG], const Sym<double> (&e)[6], double wgt) {
    double tr[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) tr[k] = e[k].xx + e[k].yy + e[k].zz;
    int q = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int l = k; l < 6; ++l) {
            const double ee = e[k].xx * e[l].xx + e[k].yy * e[l].yy + e[k].zz * e[l].zz +
                              2.0 * (e[k].yz * e[l].yz + e[k].xz * e[l].xz + e[k].xy * e[l].xy);
            acc[q] += wgt * tr[k] * tr[l];
            acc[NPAIR + q] += wgt * 2.0 * ee;
            ++q;
        }
    }
}

__device__ __forceinline__ void table_add(double *tab, int m, const double (&acc)[NG]) {
#pragma unroll
    for (int q = 0; q < NG; ++q) atomicAdd(&tab[m * NG + q], acc[q]);
}

struct GradArgs {
    const double *u, *ue;            // [6][3][N], [6][3][nX]
    const int32_t *vmat, *irr, *irr_j, *irr_lab;
    const double *irr_L, *d0is;
    int n0, n1, n2;
    int64_t N, nX, nirr;
    int nphase;
    double *partial;                 // [blocks][nphase][42]
};

template <int t>
__device__ __forceinline__ void regular_tet_strains(const double (&U)[6][8][3], Sym<double> (&e)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) v[a][i] = U[k][tet_corner(t, a)][i];
        e[k] = sym_of(kuhn_grad<t>(v));
    }
}

__device__ __forceinline__ Sym<double> unit_strain(int k) {
    double m[6] = {0, 0, 0, 0, 0, 0};
    m[k] = 1.0;
    return from_mandel<double>(m);
}

template <int t>
__device__ __forceinline__ void regular_voxel_grad(const double (&U)[6][8][3], double (&acc)[NG]) {
    Sym<double> e[6];
    regular_tet_strains<t>(U, e);
#pragma unroll
    for (int k = 0; k < 6; ++k) sym_axpy(e[k], 1.0, unit_strain(k));
    add_products(acc, e, 1.0 / 6.0);
}

__global__ __launch_bounds__(GT) void k_grad_regular(GradArgs A) {
    extern __shared__ double tab[];
    for (int q = threadIdx.x; q < A.nphase * NG; q += GT) tab[q] = 0.0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * GT;
    for (int64_t v = (int64_t)blockIdx.x * GT + threadIdx.x; v < A.N; v += stride) {
        const int m = A.vmat[v];
        if (m < 0) continue;
        const int i = (int)(v % A.n0), j = (int)((v / A.n0) % A.n1), k = (int)(v / ((int64_t)A.n0 * A.n1));
        double U[6][8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t node = wrapg(i + (c & 1), A.n0) +
                                 (int64_t)A.n0 * (wrapg(j + ((c >> 1) & 1), A.n1) + (int64_t)A.n1 * wrapg(k + (c >> 2), A.n2));
#pragma unroll
            for (int l = 0; l < 6; ++l)
#pragma unroll
                for (int d = 0; d < 3; ++d) U[l][c][d] = A.u[((int64_t)l * 3 + d) * A.N + node];
        }
        double acc[NG];
#pragma unroll
        for (int q = 0; q < NG; ++q) acc[q] = 0.0;
        regular_voxel_grad<0>(U, acc);
        regular_voxel_grad<1>(U, acc);
        regular_voxel_grad<2>(U, acc);
        regular_voxel_grad<3>(U, acc);
        regular_voxel_grad<4>(U, acc);
        regular_voxel_grad<5>(U, acc);
        table_add(tab, m, acc);
    }
    __syncthreads();
    double *out = A.partial + (int64_t)blockIdx.x * A.nphase * NG;
    for (int q = threadIdx.x; q < A.nphase * NG; q += GT) out[q] = tab[q];
}

// Cholesky factor R (lower) of a 4x4 positive semi-definite matrix; pivots
// that round to <= 0 (degenerate slivers) give zero columns.
__device__ __forceinline__ void chol4(const double (&M)[4][4], double (&R)[4][4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) R[a][b] = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = M[j][j];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < j) d -= R[j][k] * R[j][k];
        const double piv = d > 0.0 ? sqrt(d) : 0.0;
        R[j][j] = piv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i > j) {
                double s = M[i][j];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < j) s -= R[i][k] * R[j][k];
                R[i][j] = piv > 0.0 ? s / piv : 0.0;
            }
        }
    }
}

template <int t>
__device__ void irregular_tet_grad(const double (&Lc)[8], const int32_t *lab, const double (&U)[6][8][3],
                                   const double (&Q)[6][8][3], double *tab, int nphase) {
    double L[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) L[a] = Lc[tet_corner(t, a)];
    const bool anyp = L[0] > 0 || L[1] > 0 || L[2] > 0 || L[3] > 0;
    const bool anyn = L[0] < 0 || L[1] < 0 || L[2] < 0 || L[3] < 0;
    Sym<double> eF[6];
    regular_tet_strains<t>(U, eF);
#pragma unroll
    for (int k = 0; k < 6; ++k) sym_axpy(eF[k], 1.0, unit_strain(k));
    double acc[NG];
    if (!(anyp && anyn)) {
#pragma unroll
        for (int q = 0; q < NG; ++q) acc[q] = 0.0;
        add_products(acc, eF, 1.0 / 6.0);
        table_add(tab, lab[2 * t], acc);
        return;
    }
    constexpr int p0 = perm_axis(t, 0), p1 = perm_axis(t, 1), p2 = perm_axis(t, 2);
    double Mp[4][4], Mm[4][4];
    side_moments<double>(L, 1.0 / 6.0, Mp, Mm);
    // enriched gradient sums H_q per load (scaled dofs already multiplied by D0^-1/2)
    Grad<double> Hq[6];
    double q4[6][4][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) q4[k][a][i] = Q[k][tet_corner(t, a)][i];
        Hq[k] = kuhn_grad<t>(q4[k]);
    }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? 1.0 : -1.0;
        double w[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) w[a] = fabs(L[a]) - sg * L[a];
        double G[3];
        G[p0] = w[1] - w[0];
        G[p1] = w[2] - w[1];
        G[p2] = w[3] - w[2];
        double R[4][4];
        chol4(side == 0 ? Mp : Mm, R);
#pragma unroll
        for (int q = 0; q < NG; ++q) acc[q] = 0.0;
#pragma unroll
        for (int jv = 0; jv < 4; ++jv) {
            // virtual point jv: weights R[c][jv] over the four nodal strain values
            double rs = 0.0, rw = 0.0;
            double rq[6][3];
#pragma unroll
            for (int k = 0; k < 6; ++k) rq[k][0] = rq[k][1] = rq[k][2] = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                rs += R[c][jv];
                rw += R[c][jv] * w[c];
#pragma unroll
                for (int k = 0; k < 6; ++k)
#pragma unroll
                    for (int i = 0; i < 3; ++i) rq[k][i] += R[c][jv] * q4[k][c][i];
            }
            Sym<double> e[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                // sum_c R_c,jv eps_kc = rs (eps_bar + sym H_FE) + rw sym H_q + sym(rq (x) G)
                Grad<double> K;
#pragma unroll
                for (int pp = 0; pp < 3; ++pp)
#pragma unroll
                    for (int i = 0; i < 3; ++i) K.h[pp][i] = rw * Hq[k].h[pp][i] + rq[k][i] * G[pp];
                e[k] = sym_of(K);
                sym_axpy(e[k], rs, eF[k]);
            }
            add_products(acc, e, 1.0);
        }
        table_add(tab, lab[2 * t + side], acc);
    }
}

__global__ __launch_bounds__(64) void k_grad_irregular(GradArgs A) {
    extern __shared__ double tab[];
    for (int q = threadIdx.x; q < A.nphase * NG; q += 64) tab[q] = 0.0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * 64;
    for (int64_t qv = (int64_t)blockIdx.x * 64 + threadIdx.x; qv < A.nirr; qv += stride) {
        const int64_t v = A.irr[qv];
        const int i = (int)(v % A.n0), j = (int)((v / A.n0) % A.n1), k = (int)(v / ((int64_t)A.n0 * A.n1));
        double Lc[8], U[6][8][3], Q[6][8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t node = wrapg(i + (c & 1), A.n0) +
                                 (int64_t)A.n0 * (wrapg(j + ((c >> 1) & 1), A.n1) + (int64_t)A.n1 * wrapg(k + (c >> 2), A.n2));
            Lc[c] = A.irr_L[c * A.nirr + qv];
            const int jc = A.irr_j[c * A.nirr + qv];
            const double sc = jc >= 0 ? A.d0is[jc] : 0.0;
#pragma unroll
            for (int l = 0; l < 6; ++l)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    U[l][c][d] = A.u[((int64_t)l * 3 + d) * A.N + node];
                    Q[l][c][d] = jc >= 0 ? sc * A.ue[((int64_t)l * 3 + d) * A.nX + jc] : 0.0;
                }
        }
        // element labels of this voxel (rows nirr apart)
        int32_t lab[12];
#pragma unroll
        for (int q = 0; q < 12; ++q) lab[q] = A.irr_lab[q * A.nirr + qv];
        irregular_tet_grad<0>(Lc, lab, U, Q, tab, A.nphase);
        irregular_tet_grad<1>(Lc, lab, U, Q, tab, A.nphase);
        irregular_tet_grad<2>(Lc, lab, U, Q, tab, A.nphase);
        irregular_tet_grad<3>(Lc, lab, U, Q, tab, A.nphase);
        irregular_tet_grad<4>(Lc, lab, U, Q, tab, A.nphase);
        irregular_tet_grad<5>(Lc, lab, U, Q, tab, A.nphase);
    }
    __syncthreads();
    double *out = A.partial + (int64_t)blockIdx.x * A.nphase * NG;
    for (int q = threadIdx.x; q < A.nphase * NG; q += 64) out[q] = tab[q];
}

// out[p][q] = sum over blocks b (in order) of partial[b][p][q]
__global__ void k_grad_reduce(int nblocks, int nvals, const double *partial, double *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nvals) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * nvals + q];
    out[q] = s;
}

}  // namespace

// dC[nphase][2][6][6] (host), from the stored unit-load solutions.
int grad_tables(xfft_problem *p, double *dC_host) {
    const Geometry &g = p->g;
    const int np = g.nphase;
    const size_t lds = sizeof(double) * (size_t)np * NG;
    if (lds > (size_t)150 * 1024) return -1;   // EINVAL: too many phases for the LDS tables
    hipStream_t s = p->stream;
    const int nb_r = 1024, nb_i = 512;
    const int nvals = np * NG;
    double *part = nullptr, *sum = nullptr;
    if (hipMalloc(&part, sizeof(double) * (size_t)(nb_r + nb_i) * nvals) != hipSuccess) return -2;
    if (hipMalloc(&sum, sizeof(double) * 2 * nvals) != hipSuccess) { (void)hipFree(part); return -2; }
    GradArgs A;
    A.u = p->sol_u; A.ue = p->sol_ue;
    A.vmat = p->vmat; A.irr = p->irr; A.irr_j = p->irr_j; A.irr_lab = p->irr_lab;
    A.irr_L = p->t64.irr_L; A.d0is = p->t64.d0is;
    A.n0 = g.n0; A.n1 = g.n1; A.n2 = g.n2; A.N = g.N; A.nX = g.nX; A.nirr = g.nirr; A.nphase = np;
    if (lds > 65536) {
        (void)hipFuncSetAttribute((const void *)k_grad_regular, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_grad_irregular, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    A.partial = part;
    k_grad_regular<<<nb_r, GT, lds, s>>>(A);
    k_grad_reduce<<<(nvals + 255) / 256, 256, 0, s>>>(nb_r, nvals, part, sum);
    int rc = 0;
    if (g.nirr > 0) {
        A.partial = part + (size_t)nb_r * nvals;
        k_grad_irregular<<<nb_i, 64, lds, s>>>(A);
        k_grad_reduce<<<(nvals + 255) / 256, 256, 0, s>>>(nb_i, nvals, part + (size_t)nb_r * nvals, sum + nvals);
    } else if (hipMemsetAsync(sum + nvals, 0, sizeof(double) * nvals, s) != hipSuccess) {
        rc = -3;
    }
    std::vector<double> h(2 * nvals);
    if (!rc && (hipMemcpyAsync(h.data(), sum, sizeof(double) * 2 * nvals, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess))
        rc = -3;
    (void)hipFree(part);
    (void)hipFree(sum);
    if (rc) return rc;
    const double V = (double)g.N;
    for (int ph = 0; ph < np; ++ph) {
        int q = 0;
        for (int k = 0; k < 6; ++k)
            for (int l = k; l < 6; ++l, ++q) {
                const double dl = (h[ph * NG + q] + h[nvals + ph * NG + q]) / V;
                const double dm = (h[ph * NG + NPAIR + q] + h[nvals + ph * NG + NPAIR + q]) / V;
                dC_host[((ph * 2 + 0) * 6 + k) * 6 + l] = dC_host[((ph * 2 + 0) * 6 + l) * 6 + k] = dl;
                dC_host[((ph * 2 + 1) * 6 + k) * 6 + l] = dC_host[((ph * 2 + 1) * 6 + l) * 6 + k] = dm;
            }
    }
    return 0;
}

}  // namespace xfft
