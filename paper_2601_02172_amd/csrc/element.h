// Element-level device math of the X-FEM operator (Sec. 3).
//
// Uncut P1 element: constant strain eps = eps_bar + sym(grad u), stress
// sigma = lambda tr(eps) I + 2 mu eps, nodal forces V sigma g_a (eq. Kapp with
// one quadrature point, eq. A0Voxel).
//
// Cut P1 element, side s = sign(L_h) in {+1, -1}: the modified abs enrichment
// (eq. modified abs enrichment) restricted to side s is the linear function
// rho_s = sum_b lambda_b w_b with w_b = |L_b| - s L_b, so the enriched
// gradient grad N_X^a = rho_s g_a + lambda_a G_s (G_s = sum_b w_b g_b) is linear
// and the strain on the side is eps(x) = sum_c lambda_c(x) eps_c with
//   eps_c = eps_bar + sym(H_FE + w_c H_q + q_c (x) G_s),
//   H_FE = sum_a u_a (x) g_a,  H_q = sum_a q_a (x) g_a,  q_a = D0_a^-1/2 u~_a.
// The integrand of eqs. Kapp and b is therefore quadratic and is integrated
// exactly through the barycentric second moments of the side,
//   M^s_cd = int_{side s} lambda_c lambda_d dV,
// which are obtained from the subdivision along L_h = 0 (Sec. 3): every piece is
// a tetrahedron with moments V_piece / 20 (s_c s_d + sum_i B_ic B_id), B its
// vertices in barycentric coordinates and s = column sums; the complementary
// side follows from M^tet_cd = V (1 + delta_cd) / 20.  This gives the same
// element matrices as the paper's four-point rule on each piece (both are
// exact for quadratics) with one moment matrix per side instead of up to 24
// quadrature points.  Forces: with S^_d = sum_c M_cd sigma_c,
//   f_a (FE)      = (sum_d S^_d) g_a,
//   f~_a (scaled) = D0_a^-1/2 [(sum_d w_d S^_d) g_a + S^_a G_s].
#pragma once

#include "common.h"

namespace xfft {

template <typename T> struct Sym {
    T xx, yy, zz, yz, xz, xy;
};

template <typename T> __device__ __forceinline__ Sym<T> sym_zero() { return {0, 0, 0, 0, 0, 0}; }

// Start value of a sum: -0 is the exact additive identity (x + (-0) == x for
// every x, -0 included; +0 is not, since -0 + +0 = +0), so the compiler drops
// the first addition into an accumulator that starts from it.
template <typename T> __device__ __forceinline__ constexpr T acc_zero() { return -(T)0; }
template <typename T> __device__ __forceinline__ Sym<T> sym_acc_zero() {
    return {acc_zero<T>(), acc_zero<T>(), acc_zero<T>(), acc_zero<T>(), acc_zero<T>(), acc_zero<T>()};
}

// Mandel 6-vector (11,22,33,sqrt2 23,sqrt2 13,sqrt2 12) -> tensor components
template <typename T> __device__ __forceinline__ Sym<T> from_mandel(const T *m) {
    const T r = (T)0.70710678118654752440;
    return {m[0], m[1], m[2], m[3] * r, m[4] * r, m[5] * r};
}

// column p (compile-time) of a symmetric tensor
template <int P, typename T> __device__ __forceinline__ void col(const Sym<T> &s, T &a, T &b, T &c) {
    if constexpr (P == 0) { a = s.xx; b = s.xy; c = s.xz; }
    else if constexpr (P == 1) { a = s.xy; b = s.yy; c = s.yz; }
    else { a = s.xz; b = s.yz; c = s.zz; }
}

// 3x3 displacement gradient stored by columns: H[p][i] = d u_i / d x_p
template <typename T> struct Grad { T h[3][3]; };

// H = sum_a v_a (x) g_a for the Kuhn tet t with vertex vectors v[0..3] (compile-time t):
// column p0 = v1 - v0, column p1 = v2 - v1, column p2 = v3 - v2.
template <int t, typename T>
__device__ __forceinline__ Grad<T> kuhn_grad(const T (&v)[4][3]) {
    constexpr int p0 = perm_axis(t, 0), p1 = perm_axis(t, 1), p2 = perm_axis(t, 2);
    Grad<T> H;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        H.h[p0][i] = v[1][i] - v[0][i];
        H.h[p1][i] = v[2][i] - v[1][i];
        H.h[p2][i] = v[3][i] - v[2][i];
    }
    return H;
}

template <typename T>
__device__ __forceinline__ Sym<T> sym_of(const Grad<T> &H) {
    const T hf = (T)0.5;
    return {H.h[0][0], H.h[1][1], H.h[2][2],
            hf * (H.h[2][1] + H.h[1][2]), hf * (H.h[2][0] + H.h[0][2]), hf * (H.h[1][0] + H.h[0][1])};
}

template <typename T>
__device__ __forceinline__ Sym<T> hooke(const Sym<T> &e, T lam, T mu2) {
    const T tr = lam * (e.xx + e.yy + e.zz);
    return {tr + mu2 * e.xx, tr + mu2 * e.yy, tr + mu2 * e.zz, mu2 * e.yz, mu2 * e.xz, mu2 * e.xy};
}

template <typename T>
__device__ __forceinline__ void sym_axpy(Sym<T> &y, T a, const Sym<T> &x) {
    y.xx += a * x.xx; y.yy += a * x.yy; y.zz += a * x.zz;
    y.yz += a * x.yz; y.xz += a * x.xz; y.xy += a * x.xy;
}

// f[corner] += sigma g_a for the four vertices of Kuhn tet t (scaled by V beforehand)
template <int t, typename T>
__device__ __forceinline__ void kuhn_scatter(const Sym<T> &s, T (&F)[8][3]) {
    constexpr int p0 = perm_axis(t, 0), p1 = perm_axis(t, 1), p2 = perm_axis(t, 2);
    constexpr int c0 = tet_corner(t, 0), c1 = tet_corner(t, 1), c2 = tet_corner(t, 2), c3 = tet_corner(t, 3);
    T a0, b0, d0, a1, b1, d1, a2, b2, d2;
    col<p0>(s, a0, b0, d0);
    col<p1>(s, a1, b1, d1);
    col<p2>(s, a2, b2, d2);
    F[c0][0] -= a0; F[c0][1] -= b0; F[c0][2] -= d0;
    F[c1][0] += a0 - a1; F[c1][1] += b0 - b1; F[c1][2] += d0 - d1;
    F[c2][0] += a1 - a2; F[c2][1] += b1 - b2; F[c2][2] += d1 - d2;
    F[c3][0] += a2; F[c3][1] += b2; F[c3][2] += d2;
}

// ------------------------------------------------------------------ moments of the sides
template <typename T>
__device__ __forceinline__ void bary_point(T (&row)[4], int p, int q, T t) {
#pragma unroll
    for (int c = 0; c < 4; ++c) row[c] = (c == p ? (T)1 - t : (T)0) + (c == q ? t : (T)0);
}

template <typename T>
__device__ __forceinline__ T det4(const T (&B)[4][4]) {
    // cofactor expansion along the first row
    const T a = B[1][1] * (B[2][2] * B[3][3] - B[2][3] * B[3][2]) - B[1][2] * (B[2][1] * B[3][3] - B[2][3] * B[3][1])
              + B[1][3] * (B[2][1] * B[3][2] - B[2][2] * B[3][1]);
    const T b = B[1][0] * (B[2][2] * B[3][3] - B[2][3] * B[3][2]) - B[1][2] * (B[2][0] * B[3][3] - B[2][3] * B[3][0])
              + B[1][3] * (B[2][0] * B[3][2] - B[2][2] * B[3][0]);
    const T c = B[1][0] * (B[2][1] * B[3][3] - B[2][3] * B[3][1]) - B[1][1] * (B[2][0] * B[3][3] - B[2][3] * B[3][0])
              + B[1][3] * (B[2][0] * B[3][1] - B[2][1] * B[3][0]);
    const T d = B[1][0] * (B[2][1] * B[3][2] - B[2][2] * B[3][1]) - B[1][1] * (B[2][0] * B[3][2] - B[2][2] * B[3][0])
              + B[1][2] * (B[2][0] * B[3][1] - B[2][1] * B[3][0]);
    return B[0][0] * a - B[0][1] * b + B[0][2] * c - B[0][3] * d;
}

// M += moments of the piece with barycentric vertex rows B (parent volume V)
template <typename T>
__device__ __forceinline__ void add_piece(T (&M)[4][4], const T (&B)[4][4], T V) {
    const T Vs = V * fabs(det4(B)) * (T)0.05;
    T s[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] = B[0][c] + B[1][c] + B[2][c] + B[3][c];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = 0; d < 4; ++d)
            M[c][d] += Vs * (s[c] * s[d] + B[0][c] * B[0][d] + B[1][c] * B[1][d] + B[2][c] * B[2][d] + B[3][c] * B[3][d]);
}

__device__ __forceinline__ int nth_bit(unsigned m, int k) {
    for (int i = 0; i < k; ++i) m &= m - 1;
    return __ffs(m) - 1;
}

// Second moments Ms of the side of a cut element (L has both signs) that the
// subdivision builds directly (one corner tetrahedron, or the prism side);
// returns true when that is the + side.  The other side is the complement
// M^tet - Ms.
template <typename T>
__device__ bool small_side_moments(const T (&L)[4], T V, T (&Ms)[4][4]) {
    unsigned pm = 0, nm = 0, zm = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        pm |= (L[a] > (T)0) ? (1u << a) : 0u;
        nm |= (L[a] < (T)0) ? (1u << a) : 0u;
        zm |= (L[a] == (T)0) ? (1u << a) : 0u;
    }
    const int np = __popc(pm), nn = __popc(nm), nz = __popc(zm);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = 0; d < 4; ++d) Ms[c][d] = 0;
    bool small_is_pos = true;     // Ms holds the moments of the + side (else of the - side)
    auto cutp = [&](int p, int q) -> T {
        T Lp = 0, Lq = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a) { Lp = (a == p) ? L[a] : Lp; Lq = (a == q) ? L[a] : Lq; }
        return Lp / (Lp - Lq);
    };
    T B[4][4];
    if (nz == 0 && (np == 1 || nn == 1) && np + nn == 4) {
        // lone vertex: one corner tetrahedron
        const unsigned lm = (np == 1) ? pm : nm, om = (np == 1) ? nm : pm;
        small_is_pos = (np == 1);
        const int l = __ffs(lm) - 1;
        bary_point(B[0], l, -1, (T)0);
#pragma unroll
        for (int k = 0; k < 3; ++k) { const int o = nth_bit(om, k); bary_point(B[k + 1], l, o, cutp(l, o)); }
        add_piece(Ms, B, V);
    } else if (nz == 0) {
        // two and two: the + side is a prism split into three pieces
        const int p1 = nth_bit(pm, 0), p2 = nth_bit(pm, 1), n1 = nth_bit(nm, 0), n2 = nth_bit(nm, 1);
        T a0[4], a1[4], a2[4], b0[4], b1[4], b2[4];
        bary_point(a0, p1, -1, (T)0);
        bary_point(a1, p1, n1, cutp(p1, n1));
        bary_point(a2, p1, n2, cutp(p1, n2));
        bary_point(b0, p2, -1, (T)0);
        bary_point(b1, p2, n1, cutp(p2, n1));
        bary_point(b2, p2, n2, cutp(p2, n2));
#pragma unroll
        for (int c = 0; c < 4; ++c) { B[0][c] = a0[c]; B[1][c] = a1[c]; B[2][c] = a2[c]; B[3][c] = b0[c]; }
        add_piece(Ms, B, V);
#pragma unroll
        for (int c = 0; c < 4; ++c) { B[0][c] = a1[c]; B[1][c] = a2[c]; B[2][c] = b0[c]; B[3][c] = b1[c]; }
        add_piece(Ms, B, V);
#pragma unroll
        for (int c = 0; c < 4; ++c) { B[0][c] = a2[c]; B[1][c] = b0[c]; B[2][c] = b1[c]; B[3][c] = b2[c]; }
        add_piece(Ms, B, V);
        small_is_pos = true;
    } else if (nz == 1) {
        // one zero vertex: the side with a single vertex is a tetrahedron
        const unsigned lm = (np == 1) ? pm : nm, om = (np == 1) ? nm : pm;
        small_is_pos = (np == 1);
        const int l = __ffs(lm) - 1, z = __ffs(zm) - 1;
        const int o1 = nth_bit(om, 0), o2 = nth_bit(om, 1);
        bary_point(B[0], l, -1, (T)0);
        bary_point(B[1], z, -1, (T)0);
        bary_point(B[2], l, o1, cutp(l, o1));
        bary_point(B[3], l, o2, cutp(l, o2));
        add_piece(Ms, B, V);
    } else {
        // two zero vertices: both sides are tetrahedra
        const int p = __ffs(pm) - 1, n = __ffs(nm) - 1, z1 = nth_bit(zm, 0), z2 = nth_bit(zm, 1);
        bary_point(B[0], p, -1, (T)0);
        bary_point(B[1], z1, -1, (T)0);
        bary_point(B[2], z2, -1, (T)0);
        bary_point(B[3], p, n, cutp(p, n));
        add_piece(Ms, B, V);
        small_is_pos = true;
    }
    return small_is_pos;
}

// moments of both sides from the directly built side (entry of M^tet: V (1 + delta_cd) / 20)
template <typename T>
__device__ __forceinline__ void complete_sides(const T (&Ms)[4][4], bool small_is_pos, T V, T (&Mp)[4][4],
                                               T (&Mm)[4][4]) {
    const T Vt = V * (T)0.05;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const T tot = Vt * (c == d ? (T)2 : (T)1);
            Mp[c][d] = small_is_pos ? Ms[c][d] : tot - Ms[c][d];
            Mm[c][d] = small_is_pos ? tot - Ms[c][d] : Ms[c][d];
        }
}

// Second moments of both sides of a cut element (L has both signs).
template <typename T>
__device__ void side_moments(const T (&L)[4], T V, T (&Mp)[4][4], T (&Mm)[4][4]) {
    T Ms[4][4];
    const bool pos = small_side_moments<T>(L, V, Ms);
    complete_sides<T>(Ms, pos, V, Mp, Mm);
}

// barycentric gradient of vertex a of Kuhn tet t as a vector (compile-time t)
template <int t, typename T>
__device__ __forceinline__ void kuhn_g(int a, T (&g)[3]) {
    constexpr int p0 = perm_axis(t, 0), p1 = perm_axis(t, 1), p2 = perm_axis(t, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T e0 = (i == p0) ? (T)1 : (T)0, e1 = (i == p1) ? (T)1 : (T)0, e2 = (i == p2) ? (T)1 : (T)0;
        g[i] = (a == 0) ? -e0 : (a == 1) ? e0 - e1 : (a == 2) ? e1 - e2 : e2;
    }
}

// Material labels of an element: uncut -> vertex with the largest |L|; cut ->
// + side: vertex with the largest L, - side: vertex with the largest |L| among
// negative ones.  Ties go to the first vertex along the path.
template <typename T>
__device__ __forceinline__ void element_labels(const T (&L)[4], const int (&lab)[4], int &l_uncut, int &l_pos,
                                               int &l_neg, bool &multilabel) {
    T best = (T)-1, bp = (T)-1, bn = (T)-1;
    l_uncut = lab[0]; l_pos = -1; l_neg = -1;
    int fp = -1, fn = -1;
    multilabel = false;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const T v = fabs(L[a]);
        if (v > best) { best = v; l_uncut = lab[a]; }
        if (L[a] > (T)0) {
            if (L[a] > bp) { bp = L[a]; l_pos = lab[a]; }
            if (fp < 0) fp = lab[a]; else if (fp != lab[a]) multilabel = true;
        }
        if (L[a] < (T)0) {
            if (-L[a] > bn) { bn = -L[a]; l_neg = lab[a]; }
            if (fn < 0) fn = lab[a]; else if (fn != lab[a]) multilabel = true;
        }
    }
}

}  // namespace xfft
