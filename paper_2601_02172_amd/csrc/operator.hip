// Matrix-free scaled X-FEM operator (eqs. linearSystem_element, resVector).
//
// Two kernels per application, all deterministic (no atomics):
//  k_irregular  one thread per irregular voxel (a voxel with a cut element or
//               elements of different materials); evaluates its six elements
//               (cut ones by the per-side moment form of element.h) and writes
//               the eight corner forces (3 FE + 3 scaled enriched) to a buffer;
//  k_regular    z-marching LDS tile over the whole grid: every thread owns a
//               column of voxels, evaluates the six Kuhn elements of one voxel
//               per plane (or takes the buffered corner forces of an irregular
//               voxel) and the corner forces are summed per node through LDS;
//  enriched     one thread per enriched node; sums the buffered enriched
//               corner forces of its (at most eight) irregular voxels (extra
//               workgroups at the end of the k_regular launch).
#include "kernels.h"
#include <algorithm>
#include <type_traits>
#include "element.h"

namespace xfft {

namespace {

constexpr int TE = 16;          // tile edge in threads
constexpr int TO = TE - 1;      // owned nodes per tile edge
constexpr int TC = TE + 1;      // node columns per tile edge (halo on the + side)

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Position of value k (0..23: corner k / 3, component k % 3) of irregular voxel q
// in one half of the corner-force buffer: groups of 64 voxels, six rows of four
// values per voxel, rows of the 64 voxels adjacent.  The irregular kernel writes
// a whole row per lane and a wave covers a contiguous block; the regular kernel
// reads a voxel's 24 values as six 4-vectors.
__device__ __forceinline__ uint32_t cut_index(uint32_t q, int k) {
    return (((q >> 6) * 6 + (uint32_t)(k >> 2)) * 64 + (q & 63)) * 4 + (uint32_t)(k & 3);
}

// base[i] with a 32-bit byte offset (uniform base pointer + 32-bit lane offset)
template <typename P> __device__ __forceinline__ P &elem(P *base, uint32_t i) {
    using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return *reinterpret_cast<P *>(reinterpret_cast<B *>(base) + (uint32_t)(i * (uint32_t)sizeof(P)));
}

template <typename T>
struct OpArgs {
    const T *x, *xe;
    T *y, *ye;
    const double *ebar;       // [rhs][6] Mandel
    T sign;
    const Flags *flags;
    int parity;
    const int32_t *vmat, *irr, *irr_j, *irr_lab, *jlist, *enr_src;
    const T *d0is, *lame;
    const T *irr_L;           // [8][nirr] corner level set
    const T *irr_M;           // [6][10][nirr] precomputed moments of the smaller side
    T *cutbuf;
    double *partial;
    int nslots, slot0;
    double *vstress;          // [rhs][6][N] voxel-average Mandel stress, or null
    int n0, n1, n2;
    int64_t N, nX, nirr;
    int kz, tiles_x;
    int tiles_xy, reg_blocks, cut_blocks, enr_blocks;   // workgroups per right-hand side
    int nrhs;                 // right-hand sides of the launch
    int enr_slot0;            // first partial slot of the enriched gather
};

template <typename T>
__device__ __forceinline__ bool rhs_active(const OpArgs<T> &A, int r) {
    return A.flags == nullptr || A.flags[r].active[A.parity] != 0;
}

template <typename T>
__device__ __forceinline__ Sym<T> load_ebar(const double *e) {
    T m[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) m[q] = (T)e[q];
    return from_mandel<T>(m);
}

template <typename T>
__device__ __forceinline__ void add_sym(double (&acc)[7], const Sym<T> &s) {
    acc[1] += (double)s.xx; acc[2] += (double)s.yy; acc[3] += (double)s.zz;
    acc[4] += (double)s.yz; acc[5] += (double)s.xz; acc[6] += (double)s.xy;
}

template <typename T>
__device__ __forceinline__ void store_vstress(double *vs, int64_t N, int64_t v, const Sym<T> &s) {
    const double r2 = 1.41421356237309504880;
    vs[0 * N + v] = (double)s.xx; vs[1 * N + v] = (double)s.yy; vs[2 * N + v] = (double)s.zz;
    vs[3 * N + v] = r2 * (double)s.yz; vs[4 * N + v] = r2 * (double)s.xz; vs[5 * N + v] = r2 * (double)s.xy;
}

// ---------------------------------------------------------------- regular voxel: 6 Kuhn tets
// The six elements of a voxel use 12 distinct edges: 3 first edges 0 -> e_a,
// 6 middle edges e_a -> e_a + e_b and 3 last edges 7 - e_c -> 7.  The element
// with axis order (a, b, c) has displacement-gradient columns (first a, middle
// ab, last c); its stress columns are the forces of those edges (force on the
// end corner, minus on the start corner).  Corner forces are assembled from
// the 12 edge forces.  lamV, muV are lambda and mu times the element volume.
template <typename T> struct EdgeSet {
    T first[3][3], mid[3][3][3], last[3][3];   // [axis...][component]
};

template <int a, int b, int c, typename T, bool EB, bool ST>
__device__ __forceinline__ void kuhn_tet_edges(const EdgeSet<T> &E, const T (&eb)[3][3], T lamV, T muV,
                                               EdgeSet<T> &G, Sym<T> &S) {
    const T *P = E.first[a], *Q = E.mid[a][b], *R = E.last[c];
    T ea = P[a], ebb = Q[b], ec = R[c];
    T gab = Q[a] + P[b], gac = R[a] + P[c], gbc = R[b] + Q[c];
    if constexpr (EB) {
        ea += eb[a][a]; ebb += eb[b][b]; ec += eb[c][c];
        gab += (T)2 * eb[a][b]; gac += (T)2 * eb[a][c]; gbc += (T)2 * eb[b][c];
    }
    const T lt = lamV * (ea + ebb + ec);
    const T mu2 = muV + muV;
    const T saa = lt + mu2 * ea, sbb = lt + mu2 * ebb, scc = lt + mu2 * ec;
    const T sab = muV * gab, sac = muV * gac, sbc = muV * gbc;
    // column a -> first edge a (shared by (a,b,c) and (a,c,b): accumulate)
    G.first[a][a] += saa; G.first[a][b] += sab; G.first[a][c] += sac;
    // column b -> middle edge ab (used once)
    G.mid[a][b][a] = sab; G.mid[a][b][b] = sbb; G.mid[a][b][c] = sbc;
    // column c -> last edge c (shared by (a,b,c) and (b,a,c))
    G.last[c][a] += sac; G.last[c][b] += sbc; G.last[c][c] += scc;
    if constexpr (ST) {
        // tensor components by global axis
        T sx[3][3];
        sx[a][a] = saa; sx[b][b] = sbb; sx[c][c] = scc;
        sx[a][b] = sx[b][a] = sab; sx[a][c] = sx[c][a] = sac; sx[b][c] = sx[c][b] = sbc;
        S.xx += sx[0][0]; S.yy += sx[1][1]; S.zz += sx[2][2];
        S.yz += sx[1][2]; S.xz += sx[0][2]; S.xy += sx[0][1];
    }
}

template <typename T, bool EB, bool ST>
__device__ __forceinline__ void regular_voxel(const T (&U)[8][3], const T (&eb)[3][3], T lamV, T muV,
                                              T (&F)[8][3], Sym<T> &S) {
    EdgeSet<T> E, G;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            E.first[a][i] = U[1 << a][i] - U[0][i];
            E.last[a][i] = U[7][i] - U[7 ^ (1 << a)][i];
            G.first[a][i] = acc_zero<T>();
            G.last[a][i] = acc_zero<T>();
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (a != b) E.mid[a][b][i] = U[(1 << a) | (1 << b)][i] - U[1 << a][i];
        }
    }
    kuhn_tet_edges<0, 1, 2, T, EB, ST>(E, eb, lamV, muV, G, S);
    kuhn_tet_edges<0, 2, 1, T, EB, ST>(E, eb, lamV, muV, G, S);
    kuhn_tet_edges<1, 0, 2, T, EB, ST>(E, eb, lamV, muV, G, S);
    kuhn_tet_edges<1, 2, 0, T, EB, ST>(E, eb, lamV, muV, G, S);
    kuhn_tet_edges<2, 0, 1, T, EB, ST>(E, eb, lamV, muV, G, S);
    kuhn_tet_edges<2, 1, 0, T, EB, ST>(E, eb, lamV, muV, G, S);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        F[0][i] = -(G.first[0][i] + G.first[1][i] + G.first[2][i]);
        F[7][i] = G.last[0][i] + G.last[1][i] + G.last[2][i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // corner e_a: end of first a, start of middle edges ab
            T fa = G.first[a][i];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (b != a) fa -= G.mid[a][b][i];
            F[1 << a][i] = fa;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // corner 7 - e_c = e_a + e_b: end of middle edges ab and ba, start of last c
            const int a = (c + 1) % 3, b = (c + 2) % 3;
            F[7 ^ (1 << c)][i] = G.mid[a][b][i] + G.mid[b][a][i] - G.last[c][i];
        }
    }
}

// value of lane - 1 within each row of 16 lanes (DPP row_shr:1); lane 0 of a
// row receives 0.  The tile's thread (tx, ty) is lane tx + 16 (ty % 4) of its
// wave, so lane - 1 is the thread at tx - 1 for tx >= 1.
__device__ __forceinline__ float dpp_row_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ double dpp_row_shr1(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x111, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// z-marching tile kernel.  Block = 16 x 16 threads; thread (tx, ty) evaluates the
// voxel column with base (i0 - 1 + tx, j0 - 1 + ty) and owns the node column
// with the same base when tx, ty >= 1.  Node (a, b) collects corner c of the
// voxels (a - dx, b - dy): corners 0/4 from its own voxel, 1/5 from the thread
// at tx - 1, 2/6 from ty - 1 and 3/7 from (tx - 1, ty - 1).
template <typename T, bool HX, bool EB, bool ST>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && !ST) ? 5 : 1) void k_regular(OpArgs<T> A) {
    __shared__ T Dp[3][TC * TC][3];
    __shared__ T FB[3][6][TE * TE];    // row sums for the node above, one buffer per layer of the unrolled march
    __shared__ double red[4 * 7];

    // workgroups after the regular ones gather the enriched forces (they only
    // need the irregular-voxel buffer, so they fill the tail of this launch)
    const int64_t nreg = (int64_t)A.reg_blocks * A.nrhs;
    if ((int64_t)blockIdx.x >= nreg) {
        const int e = (int)(blockIdx.x - nreg), re = e / A.enr_blocks;
        if (rhs_active(A, re)) enriched_block<T, HX>(A, re, e - re * A.enr_blocks, red);
        return;
    }
    // logical block: (rhs, z chunk, tile y, tile x), x fastest
    const int64_t lb = xcd_remap(blockIdx.x, nreg);
    const int r = (int)(lb / A.reg_blocks), blk = (int)(lb % A.reg_blocks);
    if (!rhs_active(A, r)) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int tile = blk % A.tiles_xy, zc = blk / A.tiles_xy;
    const int bx = tile % A.tiles_x, by = tile / A.tiles_x;
    const int i0 = bx * TO, j0 = by * TO;
    const int k0 = zc * A.kz, k1 = min(k0 + A.kz, A.n2);
    const int n0 = A.n0, n1 = A.n1, n2 = A.n2;
    const int64_t N = A.N, plane_sz = (int64_t)n0 * n1;
    const int a = i0 - 1 + tx, b = j0 - 1 + ty;
    // tiles may wrap more than once around small grids: full modulo here, once.
    // Offsets are 32-bit from per-load base pointers (3 N values of T and the
    // corner-force buffer of one load stay below 2^32 bytes, checked at setup).
    const int aw = ((a % n0) + n0) % n0, bw = ((b % n1) + n1) % n1;
    const uint32_t N32 = (uint32_t)N, psz = (uint32_t)n0 * (uint32_t)n1;
    const uint32_t colv = (uint32_t)aw + (uint32_t)n0 * (uint32_t)bw;
    uint32_t colxy[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int col = tid + 256 * u;
        const int cx = col % TC, cy = col / TC;
        const int xi = (((i0 - 1 + cx) % n0) + n0) % n0, yi = (((j0 - 1 + cy) % n1) + n1) % n1;
        colxy[u] = (uint32_t)xi + (uint32_t)n0 * (uint32_t)yi;
    }
    const bool owner = tx >= 1 && ty >= 1 && a < n0 && b < n1;

    const T *x = HX ? A.x + (int64_t)r * 3 * N : nullptr;
    T *y = A.y + (int64_t)r * 3 * N;
    const T *cutbuf = A.cutbuf + (int64_t)r * cut_rows(A.nirr) * 48;
    T eb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if constexpr (EB) {
        const Sym<T> e = load_ebar<T>(A.ebar + 6 * r);
        eb[0][0] = e.xx; eb[1][1] = e.yy; eb[2][2] = e.zz;
        eb[1][2] = eb[2][1] = e.yz; eb[0][2] = eb[2][0] = e.xz; eb[0][1] = eb[1][0] = e.xy;
    }
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    double *vs = A.vstress ? A.vstress + (int64_t)r * 6 * N : nullptr;
    auto plane_off = [&](int kk) { return psz * (uint32_t)wrapi(kk, n2); };

    // Plane loads go through a ring of three register buffers: the loads of
    // plane kl + 3 are in flight while layer kl is computed and plane kl + 2
    // (loaded one layer earlier) is stored to LDS.  The march is unrolled by
    // three layers, so LDS slots, register buffers and exchange buffers are
    // compile-time indices.
    T R[3][2][3];
    auto fetch_plane = [&](int kk, T (&dst)[2][3]) {
        if constexpr (HX) {
            const uint32_t off = plane_off(kk);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (tid + 256 * u < TC * TC) {
                    const uint32_t node = colxy[u] + off;
                    dst[u][0] = elem(x, node);
                    dst[u][1] = elem(x, N32 + node);
                    dst[u][2] = elem(x, 2 * N32 + node);
                }
            }
        }
    };
    auto store_plane = [&](int slot, const T (&src)[2][3]) {
        if constexpr (HX) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int col = tid + 256 * u;
                if (col < TC * TC) {
                    Dp[slot][col][0] = src[u][0];
                    Dp[slot][col][1] = src[u][1];
                    Dp[slot][col][2] = src[u][2];
                }
            }
        }
    };

    fetch_plane(k0 - 1, R[0]);
    store_plane(0, R[0]);
    fetch_plane(k0, R[1]);
    store_plane(1, R[1]);
    if (k0 + 1 <= k1) fetch_plane(k0 + 1, R[2]);
    int mv[3];                       // material / irregular index of the voxel at layers kl, kl + 1, kl + 2
    mv[0] = elem(A.vmat, colv + plane_off(k0 - 1));
    mv[1] = (k0 < k1) ? elem(A.vmat, colv + plane_off(k0)) : 0;
    mv[2] = 0;
    // buffered corner forces of an irregular voxel.  With PF those of the voxel
    // one layer ahead are loaded a layer before they are used (24 more
    // registers); without it the FP32 kernel fits five waves per SIMD (86
    // registers), which hides the load latency better
    constexpr bool PF = false;
    T Fn[8][3];
    auto fetch_cut = [&](int mq) {
        const uint32_t q = (uint32_t)(-mq - 1);
        T v[24];
#pragma unroll
        for (int k4 = 0; k4 < 6; ++k4) {
            using V4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
            const V4 w = elem(reinterpret_cast<const V4 *>(cutbuf), cut_index(q, 4 * k4) >> 2);
            v[4 * k4] = w.x; v[4 * k4 + 1] = w.y; v[4 * k4 + 2] = w.z; v[4 * k4 + 3] = w.w;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) Fn[c][i] = v[3 * c + i];
    };
    if (PF && mv[0] < 0) fetch_cut(mv[0]);
    __syncthreads();

    T acc[3] = {0, 0, 0};
    // layer s (kl = k0 - 1 + s) uses LDS planes in slots sb (kl) and st (kl + 1)
    // and stores plane kl + 2 to slot sn
    auto layer = [&](auto slot_tag, int s) {
        constexpr int sb = decltype(slot_tag)::value, st = (sb + 1) % 3, sn = (sb + 2) % 3;
        const int kl = k0 - 1 + s;
        const bool more = kl + 2 <= k1, more2 = kl + 3 <= k1;
        if (more2) fetch_plane(kl + 3, R[sb]);
        mv[sn] = (kl + 2 < k1) ? elem(A.vmat, colv + plane_off(kl + 2)) : 0;
        const int m = mv[sb], mn = mv[st];
        const uint32_t vox = colv + plane_off(kl);
        T F[8][3];
        if (m < 0) {
            if (!PF) fetch_cut(m);
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) F[c][i] = Fn[c][i];
        }
        if (PF && mn < 0) fetch_cut(mn);
        if (m >= 0) {
            T U[8][3];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int col = (tx + (c & 1)) + TC * (ty + ((c >> 1) & 1));
                const int sl = (c & 4) ? st : sb;
#pragma unroll
                for (int i = 0; i < 3; ++i) U[c][i] = HX ? Dp[sl][col][i] : (T)0;
            }
            const T V = (T)(1.0 / 6.0);
            const T lamV = V * A.lame[2 * m], muV = V * A.lame[2 * m + 1];
            Sym<T> S = sym_acc_zero<T>();
            regular_voxel<T, EB, ST>(U, eb, lamV, muV, F, S);
            if (ST && owner && kl >= k0) {
                add_sym(acc7, S);
                if (vs) store_vstress(vs, N, (int64_t)vox, S);
            }
        }
        // Corner sums of node (a, b): own corner 0 (4), corner 1 (5) of the voxel
        // at a - 1 (lane tx - 1 of the same 16-lane row, moved by DPP), and the
        // row sum "corner 2 (6) + left neighbour's corner 3 (7)" of the thread
        // at b - 1, exchanged through LDS.
        T bot[3], top[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            bot[i] = F[0][i] + dpp_row_shr1(F[1][i]);
            top[i] = F[4][i] + dpp_row_shr1(F[5][i]);
            FB[sb][i][tid] = F[2][i] + dpp_row_shr1(F[3][i]);
            FB[sb][3 + i][tid] = F[6][i] + dpp_row_shr1(F[7][i]);
        }
        T dv[3] = {0, 0, 0};
        if constexpr (HX) {
#pragma unroll
            for (int i = 0; i < 3; ++i) dv[i] = Dp[sb][tx + TC * ty][i];
        }
        if (more) store_plane(sn, R[sn]);
        // one barrier per layer: the row sums rotate through three buffers, and
        // the Dp slot written next layer was last read before this barrier
        __syncthreads();
        if (owner) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bot[i] += FB[sb][i][tid - 16];
                top[i] += FB[sb][3 + i][tid - 16];
            }
            if (kl >= k0) {
                T dot = 0;                 // three terms in T, summed over the column in FP64
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const T out = A.sign * (acc[i] + bot[i]);
                    elem(y, (uint32_t)i * N32 + vox) = out;
                    if constexpr (HX) dot += out * dv[i];
                }
                acc7[0] += (double)dot;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) acc[i] = top[i];
        }
    };
    const int nlayer = k1 - k0 + 1;
    for (int s = 0; s < nlayer; s += 3) {
        layer(std::integral_constant<int, 0>{}, s);
        if (s + 1 < nlayer) layer(std::integral_constant<int, 1>{}, s + 1);
        if (s + 2 < nlayer) layer(std::integral_constant<int, 2>{}, s + 2);
    }
    __syncthreads();
    block_sum<7>(acc7, red);
    if (tid == 0) {
        double *P = A.partial + ((int64_t)r * A.nslots + A.slot0 + blk) * NPART;
#pragma unroll
        for (int q = 0; q < 7; ++q) P[q] = acc7[q];
    }
}

// ---------------------------------------------------------------- irregular voxel
// M, lab: moment and label tables (rows nirr apart, irregular voxel qv fastest).
template <int t, typename T, bool EB>
__device__ __forceinline__ void irregular_tet(const T (&Lc)[8], const T *__restrict__ M, int64_t nirr, uint32_t qv,
                                              const T (&U)[8][3], const T (&Q)[8][3],
                                              const int32_t *lab, const T *lame, const Sym<T> &eb,
                                              T (&F)[8][3], T (&Fe)[8][3], Sym<T> &S) {
    constexpr int p0 = perm_axis(t, 0), p1 = perm_axis(t, 1), p2 = perm_axis(t, 2);
    T L[4], u[4][3], q[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        L[a] = Lc[tet_corner(t, a)];
#pragma unroll
        for (int i = 0; i < 3; ++i) { u[a][i] = U[tet_corner(t, a)][i]; q[a][i] = Q[tet_corner(t, a)][i]; }
    }
    const bool anyp = L[0] > (T)0 || L[1] > (T)0 || L[2] > (T)0 || L[3] > (T)0;
    const bool anyn = L[0] < (T)0 || L[1] < (T)0 || L[2] < (T)0 || L[3] < (T)0;
    const T V = (T)(1.0 / 6.0);
    const Grad<T> HF = kuhn_grad<t>(u);
    if (!(anyp && anyn)) {
        const int m = elem(lab + (2 * t) * nirr, qv);
        Sym<T> e = sym_of(HF);
        if constexpr (EB) {
            e.xx += eb.xx; e.yy += eb.yy; e.zz += eb.zz; e.yz += eb.yz; e.xz += eb.xz; e.xy += eb.xy;
        }
        const Sym<T> s = hooke(e, V * lame[2 * m], V * (T)2 * lame[2 * m + 1]);
        kuhn_scatter<t>(s, F);
        sym_axpy(S, (T)1, s);
        return;
    }
    // Side moments: the smaller side was computed in FP64 at setup and rounded
    // once (as a difference of O(1) moments it would lose all digits in FP32);
    // the larger side is its complement.
    T Mp[4][4], Mm[4][4];
    {
        T ms[10];
#pragma unroll
        for (int e = 0; e < 10; ++e) ms[e] = elem(M + (t * 10 + e) * nirr, qv);
        const bool pos = !signbit(ms[0]);
        ms[0] = fabs(ms[0]);
        T Ms[4][4];
        int k = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = c; d < 4; ++d, ++k) Ms[c][d] = Ms[d][c] = ms[k];
        complete_sides<T>(Ms, pos, V, Mp, Mm);
    }
    const Grad<T> Hq = kuhn_grad<t>(q);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const T sg = side == 0 ? (T)1 : (T)-1;
        const int m = elem(lab + (2 * t + side) * nirr, qv);
        const T lam = lame[2 * m], mu2 = (T)2 * lame[2 * m + 1];
        T w[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) w[a] = fabs(L[a]) - sg * L[a];
        // G_s = sum_a w_a g_a with g0 = -e_p0, g1 = e_p0 - e_p1, g2 = e_p1 - e_p2, g3 = e_p2
        T G[3];
        G[p0] = w[1] - w[0];
        G[p1] = w[2] - w[1];
        G[p2] = w[3] - w[2];
        Sym<T> Sh[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) Sh[d] = sym_acc_zero<T>();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            Grad<T> K;
#pragma unroll
            for (int pp = 0; pp < 3; ++pp)
#pragma unroll
                for (int i = 0; i < 3; ++i) K.h[pp][i] = HF.h[pp][i] + w[c] * Hq.h[pp][i] + q[c][i] * G[pp];
            Sym<T> e = sym_of(K);
            if constexpr (EB) {
                e.xx += eb.xx; e.yy += eb.yy; e.zz += eb.zz; e.yz += eb.yz; e.xz += eb.xz; e.xy += eb.xy;
            }
            const Sym<T> sc = hooke(e, lam, mu2);
            const T *Mrow = side == 0 ? Mp[c] : Mm[c];
#pragma unroll
            for (int d = 0; d < 4; ++d) sym_axpy(Sh[d], Mrow[d], sc);
        }
        Sym<T> St = sym_acc_zero<T>(), Sw = sym_acc_zero<T>();
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            sym_axpy(St, (T)1, Sh[d]);
            sym_axpy(Sw, w[d], Sh[d]);
        }
        kuhn_scatter<t>(St, F);
        kuhn_scatter<t>(Sw, Fe);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int c = tet_corner(t, a);
            const Sym<T> &s = Sh[a];
            Fe[c][0] += s.xx * G[0] + s.xy * G[1] + s.xz * G[2];
            Fe[c][1] += s.xy * G[0] + s.yy * G[1] + s.yz * G[2];
            Fe[c][2] += s.xz * G[0] + s.yz * G[1] + s.zz * G[2];
        }
        sym_axpy(S, (T)1, St);
    }
}

// ST: accumulate the stress integral (criterion 0 and output passes); without
// it the partial-sum slots carry only the dot product, as in k_regular.
template <typename T, bool HX, bool EB, bool ST>
__global__ __launch_bounds__(128) void k_irregular(OpArgs<T> A) {
    __shared__ double red[2 * 7];
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r = (int)(lb / A.cut_blocks), blk = (int)(lb % A.cut_blocks);
    if (!rhs_active(A, r)) return;
    const int64_t qv = (int64_t)blk * blockDim.x + threadIdx.x;
    const uint32_t q32 = (uint32_t)qv;
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    if (qv < A.nirr) {
        const int64_t N = A.N;
        const int64_t vox = A.irr[qv];
        const int i = (int)(vox % A.n0), j = (int)((vox / A.n0) % A.n1), k = (int)(vox / ((int64_t)A.n0 * A.n1));
        T Lc[8];
        T U[8][3], Q[8][3], sc[8];
        const T *x = HX ? A.x + (int64_t)r * 3 * N : nullptr;
        const T *xe = HX ? A.xe + (int64_t)r * 3 * A.nX : nullptr;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t node = wrapi(i + (c & 1), A.n0) +
                                 (int64_t)A.n0 * (wrapi(j + ((c >> 1) & 1), A.n1) + (int64_t)A.n1 * wrapi(k + (c >> 2), A.n2));
            Lc[c] = elem(A.irr_L + c * A.nirr, q32);
            const int jc = elem(A.irr_j + c * A.nirr, q32);
            sc[c] = jc >= 0 ? A.d0is[jc] : (T)0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                U[c][d] = HX ? x[d * N + node] : (T)0;
                Q[c][d] = (HX && jc >= 0) ? sc[c] * xe[d * A.nX + jc] : (T)0;
            }
        }
        Sym<T> eb = sym_zero<T>();
        if constexpr (EB) eb = load_ebar<T>(A.ebar + 6 * r);
        const int32_t *lab = A.irr_lab;
        T F[8][3], Fe[8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) F[c][d] = Fe[c][d] = acc_zero<T>();
        Sym<T> S = sym_acc_zero<T>();
        irregular_tet<0, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        irregular_tet<1, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        irregular_tet<2, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        irregular_tet<3, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        irregular_tet<4, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        irregular_tet<5, T, EB>(Lc, A.irr_M, A.nirr, q32, U, Q, lab, A.lame, eb, F, Fe, S);
        // per-load buffer: FE corner forces [8][3][nirr], then scaled enriched ones [8][3][nirr]
        T *cb = A.cutbuf + (int64_t)r * cut_rows(A.nirr) * 48;
        T *cbe = cb + cut_rows(A.nirr) * 24;
        T vf[24], ve[24];
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                vf[3 * c + i] = F[c][i];
                ve[3 * c + i] = sc[c] * Fe[c][i];
            }
        using V4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
#pragma unroll
        for (int k4 = 0; k4 < 6; ++k4) {
            const uint32_t o = cut_index(q32, 4 * k4) >> 2;
            elem(reinterpret_cast<V4 *>(cb), o) = V4{vf[4 * k4], vf[4 * k4 + 1], vf[4 * k4 + 2], vf[4 * k4 + 3]};
            elem(reinterpret_cast<V4 *>(cbe), o) = V4{ve[4 * k4], ve[4 * k4 + 1], ve[4 * k4 + 2], ve[4 * k4 + 3]};
        }
        if constexpr (ST) {
            add_sym(acc7, S);
            if (A.vstress) store_vstress(A.vstress + (int64_t)r * 6 * N, N, vox, S);
        }
    }
    block_sum<7>(acc7, red);
    if (threadIdx.x == 0) {
        double *P = A.partial + ((int64_t)r * A.nslots + A.slot0 + blk) * NPART;
#pragma unroll
        for (int q = 0; q < 7; ++q) P[q] = acc7[q];
    }
}

// ---------------------------------------------------------------- enriched gather
// Workgroup blk (256 threads) of load r: one enriched node per thread.
template <typename T, bool HX>
__device__ __forceinline__ void enriched_block(const OpArgs<T> &A, int r, int blk, double *red) {
    const int64_t jn = (int64_t)blk * blockDim.x + threadIdx.x;
    double acc7[7] = {0, 0, 0, 0, 0, 0, 0};
    if (jn < A.nX) {
        // enr_src[j][c] = 8 * (irregular voxel) + corner, or -1: the buffered
        // corner forces that act on enriched node j
        const int4 s0 = reinterpret_cast<const int4 *>(A.enr_src)[2 * jn];
        const int4 s1 = reinterpret_cast<const int4 *>(A.enr_src)[2 * jn + 1];
        const int src[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        const T *cbe = A.cutbuf + (int64_t)r * cut_rows(A.nirr) * 48 + cut_rows(A.nirr) * 24;
        T s[3] = {0, 0, 0};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (src[c] >= 0) {
                const uint32_t q = (uint32_t)(src[c] >> 3);
                const int k = 3 * (src[c] & 7);
#pragma unroll
                for (int i = 0; i < 3; ++i) s[i] += elem(cbe, cut_index(q, k + i));
            }
        }
        T *ye = A.ye + (int64_t)r * 3 * A.nX;
        const T *xe = HX ? A.xe + (int64_t)r * 3 * A.nX : nullptr;
        double dot = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T out = A.sign * s[d];
            ye[d * A.nX + jn] = out;
            if constexpr (HX) dot += (double)out * (double)xe[d * A.nX + jn];
        }
        acc7[0] = dot;
    }
    block_sum<7>(acc7, red);
    if (threadIdx.x == 0) {
        double *P = A.partial + ((int64_t)r * A.nslots + A.enr_slot0 + blk) * NPART;
#pragma unroll
        for (int q = 0; q < 7; ++q) P[q] = acc7[q];
    }
}

// ---------------------------------------------------------------- cached voxel matrices
// Column k of the matrix of irregular voxel q: the voxel's forces for the unit
// input dof k (k < 24: FE component k % 3 of corner k / 3; k >= 24: enriched
// dof (k - 24) of the corner, entering scaled by D0^-1/2), by the moment form
// above in FP64; the outputs are the FE corner forces and the scaled enriched
// corner forces, as the irregular-voxel kernel writes them.  Column k supplies
// the rows i <= k of the packed upper triangle and the stress integral.
__global__ __launch_bounds__(128) void k_vm_build(OpArgs<double> A, double *K64, float *K32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = t / 48;
    const int k = (int)(t - q * 48);
    if (q >= A.nirr) return;
    const uint32_t q32 = (uint32_t)q;
    double Lc[8], U[8][3], Q[8][3], sc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        Lc[c] = elem(A.irr_L + c * A.nirr, q32);
        const int jc = elem(A.irr_j + c * A.nirr, q32);
        sc[c] = jc >= 0 ? A.d0is[jc] : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            U[c][d] = (k < 24 && 3 * c + d == k) ? 1.0 : 0.0;
            Q[c][d] = (k >= 24 && 3 * c + d == k - 24) ? sc[c] : 0.0;
        }
    }
    const Sym<double> eb = sym_zero<double>();
    double F[8][3], Fe[8][3];
#pragma unroll
    for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) F[c][d] = Fe[c][d] = acc_zero<double>();
    Sym<double> S = sym_acc_zero<double>();
    irregular_tet<0, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    irregular_tet<1, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    irregular_tet<2, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    irregular_tet<3, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    irregular_tet<4, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    irregular_tet<5, double, false>(Lc, A.irr_M, A.nirr, q32, U, Q, A.irr_lab, A.lame, eb, F, Fe, S);
    double *k64 = K64 + q * VM_STRIDE;
    float *k32 = K32 ? K32 + q * VM_STRIDE : nullptr;
#pragma unroll
    for (int i = 0; i < 48; ++i) {
        if (i <= k) {
            const int c = (i < 24 ? i : i - 24) / 3, d = (i < 24 ? i : i - 24) % 3;
            const double v = i < 24 ? F[c][d] : sc[c] * Fe[c][d];
            k64[vm_row(i) + k] = v;
            if (k32) k32[vm_row(i) + k] = (float)v;
        }
    }
    const double st[6] = {S.xx, S.yy, S.zz, S.yz, S.xz, S.xy};
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        k64[VM_KP + 48 * m + k] = st[m];
        if (k32) k32[VM_KP + 48 * m + k] = (float)st[m];
    }
    if (k < VM_KP - VM_K) {
        k64[VM_K + k] = 0.0;
        if (k32) k32[VM_K + k] = 0.0f;
    }
}

template <typename T> struct VmArgs {
    const T *x, *xe;          // inputs of load 0; loads 3 N / 3 nX apart
    T *cutbuf;                // corner-force buffer of load 0
    const T *K;               // [nirr][VM_STRIDE]
    const int32_t *irr, *irr_j;
    const Flags *flags;
    int parity;
    double *partial;
    int nslots, slot0;
    int n0, n1, n2;
    int64_t N, nX, nirr;
    int nrhs;
};

// Index data of irregular voxel q for the cached-matrix kernel, loaded two
// voxels ahead of use: its voxel (lanes < 24 and >= 48) or the enriched index
// of the lane's corner (lanes 24..47).  The address is selected, not branched
// on, so that no control-flow join waits for the load.
template <typename T>
__device__ __forceinline__ int vm_index(const VmArgs<T> &A, int64_t q, int lane, int c) {
    const bool enr = lane >= 24 && lane < 48;
    const uintptr_t a = (uintptr_t)(A.irr + q), b = (uintptr_t)(A.irr_j + (enr ? c : 0) * A.nirr + q);
    return *reinterpret_cast<const int32_t *>(enr ? b : a);
}

// Loads of irregular voxel q: this lane's share of the packed matrix (kreg)
// and its input dof of every load (xreg; lanes < 48; zero where the dof does
// not exist or the load is inactive).  Every load is issued unconditionally
// from a valid address (the last lanes repeat the final matrix vector; lanes
// without an input read node 0 of load 0) and validity is applied when the
// values are used, so the arrays stay in registers and nothing waits here.
template <typename T, typename V, int NR, int NV, int NVL>
__device__ __forceinline__ void vm_fetch(const VmArgs<T> &A, int64_t q, int idx, int lane, int c, int d,
                                         const bool (&act)[NR], V (&kreg)[NVL], T (&xreg)[NR], bool (&xok)[NR]) {
    const V *Kq = reinterpret_cast<const V *>(A.K + q * VM_STRIDE);
#pragma unroll
    for (int u = 0; u < NVL; ++u) kreg[u] = Kq[min(lane + 64 * u, NV - 1)];
    const bool fe = lane < 24, en = lane >= 24 && lane < 48 && idx >= 0;
    const int vox = fe ? idx : 0;
    const int vi = vox % A.n0, vj = (vox / A.n0) % A.n1, vk = vox / (A.n0 * A.n1);
    const int cc = fe ? c : 0;
    const int64_t node = wrapi(vi + (cc & 1), A.n0) +
                         (int64_t)A.n0 * (wrapi(vj + ((cc >> 1) & 1), A.n1) + (int64_t)A.n1 * wrapi(vk + (cc >> 2), A.n2));
    const uintptr_t pf = (uintptr_t)(A.x + (fe ? (int64_t)d * A.N + node : 0));
    const uintptr_t pe = (uintptr_t)(A.xe + (en ? (int64_t)d * A.nX + idx : 0));
    const T *src = reinterpret_cast<const T *>(en ? pe : pf);
    const int64_t stride = en ? 3 * A.nX : 3 * A.N;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        xok[r] = act[r] && (fe || en);
        xreg[r] = src[(xok[r] ? r : 0) * stride];
    }
}

// 16-byte native vectors (HIP's float4 / double2 are unions, which keep arrays of
// them in scratch memory)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

// One wave per workgroup, walking a contiguous chunk of irregular voxels; every
// active load of the launch (up to VM_MAXR) at once, so each voxel's matrix is
// read once for all loads.  Lane i < 48 owns row i (output dof i), lanes
// 48..53 the stress rows (with the stress integral).  The matrix and the 48
// inputs of each load are staged in LDS; those of the next voxel are loaded
// into registers while the current one is computed.  Outputs go to the
// corner-force buffer exactly as the moment-form kernel writes them.
template <typename T, int NR, bool ST>
__global__ __launch_bounds__(64) void k_irregular_vm(VmArgs<T> A) {
    constexpr int KN = ST ? VM_STRIDE : VM_KP;
    using V = typename std::conditional<sizeof(T) == 4, vf4, vd2>::type;
    constexpr int PER_V = 16 / sizeof(T);
    constexpr int NV = KN / PER_V, NVL = (NV + 63) / 64;     // vectors per voxel, per lane
    __shared__ V Ks4[NV];
    __shared__ V Xs4[48][8 / PER_V];          // the inputs of dof j, loads in order (padded to 8)
    const int lane = threadIdx.x;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t chunk = (A.nirr + gridDim.x - 1) / gridDim.x;
    const int64_t q0 = blk * chunk, q1 = min(q0 + chunk, A.nirr);
    const T *Ks = reinterpret_cast<const T *>(Ks4);
    T *Xs = reinterpret_cast<T *>(Xs4);
    bool act[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) act[r] = r < A.nrhs && (A.flags == nullptr || A.flags[r].active[A.parity] != 0);
    double sacc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) sacc[r] = 0.0;
    const int i = lane < 48 ? lane : 47;
    const int Ri = vm_row(i);
    const int m = lane - 48;                        // stress row of lanes 48..53
    const int kk = lane < 24 ? lane : lane - 24;    // corner-major dof of the lane's input and output
    const int c = kk / 3, d = kk - 3 * c;
    V kreg[NVL];
    T xreg[NR];
    bool xok[NR];
    int idx_next = 0;
    if (q0 < q1) {
        vm_fetch<T, V, NR, NV, NVL>(A, q0, vm_index(A, q0, lane, c), lane, c, d, act, kreg, xreg, xok);
        if (q0 + 1 < q1) idx_next = vm_index(A, q0 + 1, lane, c);
    }
    // The workgroup is one wave and the LDS accesses of a wave complete in
    // order, so the hand-over through LDS needs only a compiler-level wave
    // barrier; a workgroup barrier would also wait for the prefetch loads.
    // Stores and loads share one in-order counter: a voxel's outputs are
    // stored one step later, before the next prefetch is issued, so that
    // waiting for the prefetch never waits for stores issued just before it.
    T ylast[NR];
    int64_t qlast = -1;
    const int64_t half = cut_rows(A.nirr) * 24;
    for (int64_t q = q0; q < q1; ++q) {
        __builtin_amdgcn_wave_barrier();            // the previous voxel's LDS reads come first
#pragma unroll
        for (int u = 0; u < NVL; ++u)
            if (lane + 64 * u < NV) Ks4[lane + 64 * u] = kreg[u];
        if (lane < 48) {
#pragma unroll
            for (int r = 0; r < NR; ++r) Xs[8 * lane + r] = xok[r] ? xreg[r] : (T)0;
        }
        __builtin_amdgcn_wave_barrier();
        if (qlast >= 0 && lane < 48) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (act[r]) {
                    T *cb = A.cutbuf + (int64_t)r * cut_rows(A.nirr) * 48 + (lane < 24 ? 0 : half);
                    elem(cb, cut_index((uint32_t)qlast, kk)) = ylast[r];
                }
            }
        }
        // the next voxel's loads (its index data arrived during this voxel's
        // predecessor) and the index data of the one after stay in flight
        // while this voxel is computed
        if (q + 1 < q1) {
            vm_fetch<T, V, NR, NV, NVL>(A, q + 1, idx_next, lane, c, d, act, kreg, xreg, xok);
            if (q + 2 < q1) idx_next = vm_index(A, q + 2, lane, c);
        }
        // lanes < 48: matrix row i; lanes 48..53 (with the stress integral):
        // stress row m -- one loop, the lanes differ only in their address
        if (lane < (ST ? 54 : 48)) {
            T y[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) y[r] = acc_zero<T>();
            // eight columns per step keep the loads in flight without holding
            // the whole matrix row in registers
#pragma unroll 1
            for (int j0 = 0; j0 < 48; j0 += 8) {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int j = j0 + jj;
                    const int ka = lane < 48 ? ((j < i) ? vm_row(j) + i : Ri + j) : VM_KP + 48 * m + j;
                    const T kv = Ks[ka];
                    T xv[8];
#pragma unroll
                    for (int u = 0; u < (NR + PER_V - 1) / PER_V; ++u) {
                        const V w = Xs4[j][u];
#pragma unroll
                        for (int e = 0; e < PER_V; ++e) xv[PER_V * u + e] = w[e];
                    }
#pragma unroll
                    for (int r = 0; r < NR; ++r) y[r] += kv * xv[r];
                }
            }
            if (lane < 48) {
#pragma unroll
                for (int r = 0; r < NR; ++r) ylast[r] = y[r];
                qlast = q;
            } else {
#pragma unroll
                for (int r = 0; r < NR; ++r) sacc[r] += (double)y[r];
            }
        }
    }
    if (qlast >= 0 && lane < 48) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (act[r]) {
                T *cb = A.cutbuf + (int64_t)r * cut_rows(A.nirr) * 48 + (lane < 24 ? 0 : half);
                elem(cb, cut_index((uint32_t)qlast, kk)) = ylast[r];
            }
        }
    }
    // partial sums of the workgroup: no dot product; the stress integral by lanes 48..53
    if (lane >= 48 && m < 7) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < A.nrhs) {
                double *P = A.partial + ((int64_t)r * A.nslots + A.slot0 + blk) * NPART;
                P[m < 6 ? 1 + m : 0] = (ST && m < 6) ? sacc[r] : 0.0;
            }
        }
    }
}

template <typename T, int NR>
void launch_vm(const VmArgs<T> &A, unsigned grid, bool stress, hipStream_t s) {
    if (stress) k_irregular_vm<T, NR, true><<<grid, 64, 0, s>>>(A);
    else k_irregular_vm<T, NR, false><<<grid, 64, 0, s>>>(A);
}

}  // namespace

template <typename T>
void launch_operator_ws(xfft_problem *p, const Tables<T> &tb, const T *x, const T *xe, T *y, T *ye,
                        const double *ebar, bool use_ebar, T sign, int nrhs, const Flags *flags, int parity,
                        double *vstress, hipStream_t s, bool stress, T *cutbuf, double *partial, bool allow_vm) {
    const Geometry &g = p->g;
    const SlotLayout &L = p->slots;
    OpArgs<T> A;
    A.x = x; A.xe = xe; A.y = y; A.ye = ye;
    A.ebar = ebar; A.sign = sign; A.flags = flags; A.parity = parity;
    A.vmat = p->vmat; A.irr = p->irr; A.irr_j = p->irr_j; A.irr_lab = p->irr_lab; A.jlist = p->jlist;
    A.enr_src = p->enr_src;
    A.irr_L = tb.irr_L; A.irr_M = tb.irr_M; A.d0is = tb.d0is; A.lame = tb.lame;
    A.cutbuf = cutbuf; A.partial = partial; A.nslots = p->nslots;
    A.vstress = vstress;
    A.n0 = g.n0; A.n1 = g.n1; A.n2 = g.n2; A.N = g.N; A.nX = g.nX; A.nirr = g.nirr;
    A.kz = L.kz; A.tiles_x = L.tiles_x;
    A.tiles_xy = L.tiles_x * L.tiles_y; A.reg_blocks = L.tiles_x * L.tiles_y * L.zchunks; A.cut_blocks = L.cut_n;
    A.enr_blocks = L.enr_n;
    A.nrhs = nrhs;
    A.enr_slot0 = L.enr0;
    const bool hx = x != nullptr;
    // cached voxel matrices: operator applications without macro strain and
    // voxel stresses (the CG iterations), up to VM_MAXR loads per launch
    const T *vmK = sizeof(T) == 8 ? reinterpret_cast<const T *>(p->vm64) : reinterpret_cast<const T *>(p->vm32);
    const bool vm = allow_vm && g.nirr > 0 && hx && !use_ebar && !vstress && nrhs <= VM_MAXR && vmK &&
                    p->vm_valid && p->vm_on[sizeof(T) == 8 ? 1 : 0];
    p->last_op_vm = vm;
    if (vm) {
        VmArgs<T> V;
        V.x = x; V.xe = xe; V.cutbuf = cutbuf; V.K = vmK; V.irr = p->irr; V.irr_j = p->irr_j;
        V.flags = flags; V.parity = parity; V.partial = partial; V.nslots = p->nslots; V.slot0 = L.vm0;
        V.n0 = g.n0; V.n1 = g.n1; V.n2 = g.n2; V.N = g.N; V.nX = g.nX; V.nirr = g.nirr; V.nrhs = nrhs;
        const unsigned grid = (unsigned)L.vm_n;
        xfft_prof_mark(p, -1, s);
        if (nrhs == 1) launch_vm<T, 1>(V, grid, stress, s);
        else if (nrhs == 2) launch_vm<T, 2>(V, grid, stress, s);
        else if (nrhs == 3) launch_vm<T, 3>(V, grid, stress, s);
        else launch_vm<T, 6>(V, grid, stress, s);
        xfft_prof_mark(p, K_IRREGULAR + (sizeof(T) == 8 ? K_COUNT : 0), s);
    } else if (g.nirr > 0) {
        A.slot0 = L.cut0;
        dim3 grid((unsigned)L.cut_n * nrhs, 1);
        xfft_prof_mark(p, -1, s);
        if (hx && use_ebar) k_irregular<T, true, true, true><<<grid, 128, 0, s>>>(A);
        else if (hx && stress) k_irregular<T, true, false, true><<<grid, 128, 0, s>>>(A);
        else if (hx) k_irregular<T, true, false, false><<<grid, 128, 0, s>>>(A);
        else if (use_ebar) k_irregular<T, false, true, true><<<grid, 128, 0, s>>>(A);
        else k_irregular<T, false, false, false><<<grid, 128, 0, s>>>(A);
        xfft_prof_mark(p, K_IRREGULAR + (sizeof(T) == 8 ? K_COUNT : 0), s);
    }
    {
        A.slot0 = L.fe0;
        if (g.nX == 0) A.enr_blocks = 0;
        dim3 grid((unsigned)(L.tiles_x * L.tiles_y * L.zchunks + A.enr_blocks) * nrhs, 1);
        xfft_prof_mark(p, -1, s);
        if (hx && use_ebar) k_regular<T, true, true, true><<<grid, 256, 0, s>>>(A);
        else if (hx && stress) k_regular<T, true, false, true><<<grid, 256, 0, s>>>(A);
        else if (hx) k_regular<T, true, false, false><<<grid, 256, 0, s>>>(A);
        else if (use_ebar) k_regular<T, false, true, true><<<grid, 256, 0, s>>>(A);
        else k_regular<T, false, false, false><<<grid, 256, 0, s>>>(A);
        xfft_prof_mark(p, K_REGULAR + (sizeof(T) == 8 ? K_COUNT : 0), s);
    }
}

template <typename T>
void launch_operator(xfft_problem *p, Work<T> &w, const Tables<T> &tb, const T *x, const T *xe, T *y, T *ye,
                     bool use_ebar, T sign, int nrhs, const Flags *flags, int parity, double *vstress,
                     hipStream_t s, bool stress) {
    launch_operator_ws<T>(p, tb, x, xe, y, ye, p->ebar, use_ebar, sign, nrhs, flags, parity, vstress, s, stress,
                          w.cutbuf, p->partial, true);
}

// Cached voxel matrices of the current moduli for the requested precisions
// (FP64 built by the moment form, FP32 rounded once from it).  0, or -2 when
// the allocation fails (nothing is kept then), -3 on a launch error.
int build_voxel_matrices(xfft_problem *p, bool fp32, bool fp64) {
    const Geometry &g = p->g;
    if (g.nirr == 0) return 0;
    const size_t n = (size_t)g.nirr * VM_STRIDE;
    if (fp64 && !p->vm64 && hipMalloc(&p->vm64, n * sizeof(double)) != hipSuccess) { p->vm64 = nullptr; return -2; }
    if (fp32 && !p->vm32 && hipMalloc(&p->vm32, n * sizeof(float)) != hipSuccess) { p->vm32 = nullptr; return -2; }
    // the FP32 table is rounded from the FP64 one: build FP64 in a temporary when only FP32 is kept
    double *k64 = p->vm64;
    bool tmp = false;
    if (!k64) {
        if (hipMalloc(&k64, n * sizeof(double)) != hipSuccess) return -2;
        tmp = true;
    }
    OpArgs<double> A{};
    A.irr_j = p->irr_j; A.irr_lab = p->irr_lab; A.irr_L = p->t64.irr_L; A.irr_M = p->t64.irr_M;
    A.d0is = p->t64.d0is; A.lame = p->t64.lame; A.nirr = g.nirr;
    const int64_t nt = g.nirr * 48;
    k_vm_build<<<(unsigned)((nt + 127) / 128), 128, 0, p->stream>>>(A, k64, p->vm32);
    const bool ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(p->stream) == hipSuccess;
    if (tmp) (void)hipFree(k64);
    if (!ok) return -3;
    p->vm_valid = true;
    return 0;
}

void free_voxel_matrices(xfft_problem *p) {
    if (p->vm64) (void)hipFree(p->vm64);
    if (p->vm32) (void)hipFree(p->vm32);
    p->vm64 = nullptr;
    p->vm32 = nullptr;
    p->vm_valid = false;
    p->vm_on[0] = p->vm_on[1] = false;
}

template void launch_operator_ws<double>(xfft_problem *, const Tables<double> &, const double *, const double *,
                                         double *, double *, const double *, bool, double, int, const Flags *, int,
                                         double *, hipStream_t, bool, double *, double *, bool);
template void launch_operator<double>(xfft_problem *, Work<double> &, const Tables<double> &, const double *,
                                      const double *, double *, double *, bool, double, int, const Flags *, int,
                                      double *, hipStream_t, bool);
template void launch_operator<float>(xfft_problem *, Work<float> &, const Tables<float> &, const float *,
                                     const float *, float *, float *, bool, float, int, const Flags *, int, double *,
                                     hipStream_t, bool);

void set_depth(SlotLayout &L, const Geometry &g, int kz) {
    L.kz = kz;
    L.zchunks = (g.n2 + kz - 1) / kz;
    L.fe_n = L.tiles_x * L.tiles_y * L.zchunks;
}

SlotLayout slot_layout(const Geometry &g) {
    SlotLayout L{};
    L.tiles_x = (g.n0 + TO - 1) / TO;
    L.tiles_y = (g.n1 + TO - 1) / TO;
    // planes per block: every block recomputes one halo layer, so keep kz >= 8
    // unless the grid would be left with fewer than ~1024 blocks per load (the
    // autotuner may change it later, within the reserved slots of depth 4)
    int kz = 16;
    while (kz > 8 && (int64_t)L.tiles_x * L.tiles_y * ((g.n2 + kz - 1) / kz) < 1024) kz /= 2;
    while (kz > 4 && (int64_t)L.tiles_x * L.tiles_y * ((g.n2 + kz - 1) / kz) < 256) kz /= 2;
    int at = 0;
    L.fe0 = at;
    L.fe_cap = L.tiles_x * L.tiles_y * ((g.n2 + 3) / 4);
    at += L.fe_cap;
    set_depth(L, g, kz);
    L.cut0 = at; L.cut_n = (int)((g.nirr + 127) / 128); at += L.cut_n;
    L.enr0 = at; L.enr_n = (int)((g.nX + 255) / 256); at += L.enr_n;
    L.vm0 = at; L.vm_n = (int)std::min<int64_t>((g.nirr + VM_VPB - 1) / VM_VPB, VM_GRID); at += L.vm_n;
    L.grn0 = at; L.grn_n = 0; // filled by the FFT planner
    L.total = at;
    return L;
}

}  // namespace xfft
