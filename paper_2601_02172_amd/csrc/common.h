// Internal declarations of the X-FFT GPU library (gfx950).
//
// Geometry conventions of the device code (voxel units, h = 1):
//   node (i, j, k) -> flat index i + n0 * (j + n1 * k), periodic;
//   voxel (i, j, k) has corners (i + dx, j + dy, k + dz), corner code
//   c = dx | dy << 1 | dz << 2;
//   the six P1 elements of a voxel (Sec. 3) are the Kuhn tetrahedra that share
//   the diagonal corner 0 -> corner 7: for an axis permutation (p0, p1, p2) the
//   path 0 -> e_p0 -> e_p0 + e_p1 -> (1, 1, 1).  Barycentric gradients along the
//   path are -e_p0, e_p0 - e_p1, e_p1 - e_p2, e_p2 and the volume is 1/6.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

namespace xfft {

// ------------------------------------------------------------------ Kuhn table
// permutations in lexicographic order; PERM[t][s] = axis of step s
__host__ __device__ constexpr int perm_axis(int t, int s) {
    // (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0)
    return (t == 0) ? (s == 0 ? 0 : s == 1 ? 1 : 2)
         : (t == 1) ? (s == 0 ? 0 : s == 1 ? 2 : 1)
         : (t == 2) ? (s == 0 ? 1 : s == 1 ? 0 : 2)
         : (t == 3) ? (s == 0 ? 1 : s == 1 ? 2 : 0)
         : (t == 4) ? (s == 0 ? 2 : s == 1 ? 0 : 1)
         :            (s == 0 ? 2 : s == 1 ? 1 : 0);
}
// corner code of vertex v (0..3) of tet t
__host__ __device__ constexpr int tet_corner(int t, int v) {
    return v == 0 ? 0
         : v == 1 ? (1 << perm_axis(t, 0))
         : v == 2 ? ((1 << perm_axis(t, 0)) | (1 << perm_axis(t, 1)))
         : 7;
}

// ------------------------------------------------------------------ complex
template <typename T> struct cpx { T x, y; };

template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }

// Workgroups of a dispatch are handed to the 8 XCDs of the chip round robin
// (linear id mod 8), and each XCD has its own L2.  Giving every XCD one
// contiguous range of logical ids keeps neighbouring tiles, which read the same
// cache lines, on the same L2.  Bijective on [0, nb).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    constexpr int NXCD = 8;
    const int64_t q = nb / NXCD, rem = nb % NXCD;
    const int64_t x = b % NXCD, slot = b / NXCD;
    return x < rem ? x * (q + 1) + slot : rem * (q + 1) + (x - rem) * q + slot;
}

// ------------------------------------------------------------------ FFT plan
struct FftPlan {
    int n;            // line length
    int nstages;
    int radix[16];    // radices applied in order (4, 2, 3)
};
FftPlan make_plan(int n);

// ------------------------------------------------------------------ block reduction
// Sums NV doubles over the block; result valid in thread 0. red must hold
// NV * (blockDim.x / 64) doubles of shared memory.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        v[q] = s;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[wave * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w * NV + q];
            v[q] = s;
        }
    }
}

// ------------------------------------------------------------------ problem
constexpr int NPART = 8;   // doubles per partial-sum slot: [0] dot, [1..6] stress integral

// Row stride of the half spectrum in the layout of the separate x, y and z
// passes: nh = n0 / 2 + 1 rounded up to a multiple of 8 values.
inline int spec_row_stride(int nh) { return (nh + 7) & ~7; }

struct Geometry {
    int n0, n1, n2, nh;     // nh = n0 / 2 + 1
    int64_t N;              // nodes = voxels
    int64_t nX;             // enriched nodes
    int64_t nirr;           // irregular voxels
    int nphase;
};

// Per-precision device tables.
template <typename T> struct Tables {
    T *lame = nullptr;       // [nphase][2]
    T *d0is = nullptr;       // [nX] D0^-1/2
    // Tables of the irregular voxels are stored with the voxel index fastest
    // ([row][nirr]), so that the lanes of a wave access consecutive words.
    T *irr_L = nullptr;      // [8][nirr] snapped corner level set of irregular voxels
    // [6][10][nirr] moments of the smaller side of each cut Kuhn tet of the
    // irregular voxels (upper triangle; the sign bit of entry 0 marks the - side),
    // computed in FP64 and rounded once
    T *irr_M = nullptr;
    cpx<T> *tw[3] = {nullptr, nullptr, nullptr};   // twiddles exp(-2 pi i t / n_axis)
    cpx<T> *tws[3] = {nullptr, nullptr, nullptr};  // stage-major twiddles of the compile-time LDS FFT
    T *half[3] = {nullptr, nullptr, nullptr};      // [n_axis][2]: sin, cos of pi k / n_axis
};

// Work fields of one precision for up to `cap` right-hand sides.
template <typename T> struct Work {
    int cap = 0;
    T *u = nullptr, *f = nullptr, *d = nullptr, *z = nullptr;          // [cap][3][N]
    T *ue = nullptr, *fe = nullptr, *de = nullptr, *ze = nullptr;      // [cap][3][nX]
    cpx<T> *spec = nullptr;                                            // [cap][3][n2][n1][nh]
    // [cap][2][cut_rows(nirr) / 64][6][64][4]: FE, then scaled enriched corner
    // forces of the irregular voxels, 24 values (corner-major, xyz) per voxel in
    // groups of 64 voxels, four values per row (see cut_index in operator.hip)
    T *cutbuf = nullptr;
};

// irregular voxels rounded up to whole groups of 64 (corner-force buffer)
__host__ __device__ inline int64_t cut_rows(int64_t nirr) { return (nirr + 63) & ~(int64_t)63; }

// Cached voxel matrices (Sec. 3, caching strategy): per irregular voxel the
// scaled 48 x 48 element matrix of the voxel (8 corners x (3 FE + 3 scaled
// enriched dofs), symmetric) as its packed upper triangle, row a holding
// columns a..47 at vm_row(a) + b, then six rows of 48 giving the voxel's stress
// integral (tensor components xx, yy, zz, yz, xz, xy) per unit dof.
constexpr int VM_K = 1176;        // packed upper triangle
constexpr int VM_KP = 1184;       // start of the stress rows (padded to 16 values)
constexpr int VM_STRIDE = 1472;   // values per voxel
constexpr int VM_VPB = 4;         // fewest voxels per (one-wave) workgroup of the cached-matrix kernel
constexpr int VM_GRID = 4096;     // most workgroups of a launch (each walks a contiguous chunk of voxels)
constexpr int VM_MAXR = 6;        // loads per launch of the cached-matrix kernel
__host__ __device__ constexpr int vm_row(int a) { return 47 * a - a * (a - 1) / 2; }

// Partial-sum slot layout per right-hand side.
struct SlotLayout {
    int fe0, fe_n;      // regular-voxel operator blocks at the current depth kz
    int fe_cap;         // slots reserved for the regular-voxel blocks (depth 4)
    int cut0, cut_n;    // irregular-voxel blocks (moment form)
    int enr0, enr_n;    // enriched gather blocks
    int vm0, vm_n;      // irregular-voxel blocks of the cached voxel matrices (right after the enriched ones)
    int grn0, grn_n;    // Green (z pass) blocks
    int eu0, eu_n;      // enriched residual blocks
    int total;
    int kz;             // planes per operator block
    int tiles_x, tiles_y, zchunks;
};

struct Scalars {           // per right-hand side, device resident
    double res2, res2_0, alpha, beta;
    double sigma[6];
    double tol;            // tolerance of eq. stoppingCriterion (criterion 0)
    double tol_inner;      // residual reduction of an inner refinement solve (criterion 1)
    double s0;             // step size of eq. stepsize (schemes other than linear CG)
    double alpha_lag;      // Barzilai-Borwein: step of the next iteration (0: none yet)
};

struct Flags {
    int active[2];         // parity-buffered "iteration runs" flag
    int iters;
    int conv;
    int breakdown;
    int pad[3];            // pad[0]: outer (refinement) loop converged
};

// Kernel classes timed by the profiling hook (order of xfft_profile's output).
enum KernelId {
    K_IRREGULAR = 0, K_REGULAR, K_ENRICHED, K_FFT_X_FWD, K_FFT_Y_FWD, K_FFT_Z_GREEN, K_FFT_Y_INV, K_FFT_X_INV,
    K_ENR_UPDATE, K_ENR_FINAL, K_SCALARS, K_COUNT
};

}  // namespace xfft

struct xfft_problem;
// Records an event after a kernel launch when profiling is on (no-op otherwise).
void xfft_prof_mark(xfft_problem *p, int kernel_id, hipStream_t s);

// The opaque handle.
struct xfft_problem {
    xfft::Geometry g;
    double h = 1.0;
    double len[3];
    int device = 0;
    int num_cu = 256;         // compute units of the device (persistent grids)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // options
    double rtol, snap_eps, d0_scale, inner_rtol;
    int maxit, precision, batch, check_every;
    int scheme = 0;        // XFFT_LCG, XFFT_NLCG, XFFT_BB or XFFT_BASIC
    int p1 = 0;            // 1: voxel-segmented P1 discretisation (no enrichment)
    // geometry (device)
    double *Ls = nullptr;          // snapped level set, voxel units [N]
    int32_t *phase = nullptr;      // [N]
    int32_t *vmat = nullptr;       // [N] material (>= 0) or -(irregular index + 1)
    int32_t *irr = nullptr;        // [nirr] voxel of each irregular voxel
    int32_t *irr_j = nullptr;      // [8][nirr] enriched index per corner or -1
    int32_t *irr_lab = nullptr;    // [6][2][nirr] element labels: uncut (both) or (+ side, - side)
    int32_t *jlist = nullptr;      // [nX]
    int32_t *enr_src = nullptr;    // [nX][8] 8 * irregular voxel + corner feeding enriched node j, or -1
    double *d0 = nullptr;          // [nX]
    int64_t n_cut_elements = 0, n_multilabel = 0;
    std::vector<double> lame_host;
    xfft::Tables<double> t64;
    xfft::Tables<float> t32;
    xfft::FftPlan plan[3];
    xfft::SlotLayout slots;
    // work space
    xfft::Work<double> w64;
    xfft::Work<float> w32;
    double *partial = nullptr;     // [cap][nslots][NPART]
    double *sum7 = nullptr;        // [cap][7] sums of the output pass
    bool sigma_ready = false;      // last solve_block left the exact <sigma> of its iterate in scal
    int part_cap = 0, nslots = 0;
    xfft::Scalars *scal = nullptr; // [cap]
    xfft::Flags *flags = nullptr;  // [cap]
    double *ebar = nullptr;        // [cap][6]
    int *host_flags = nullptr;     // pinned mirror for polling
    int scal_cap = 0;
    // solutions of the last solve (FP64, voxel units) for gradients
    double *sol_u = nullptr, *sol_ue = nullptr;
    int sol_nload = 0;
    bool sol_unit_basis = false;
    // sol_u / sol_ue hold finite unit-load solutions of an earlier solve (any
    // moduli): the start of a warm-started unit-load solve
    bool sol_stored = false;
    bool warm_start = false;
    double seconds_setup = 0.0, seconds_solve = 0.0;
    // captured CG iterations (replayed as one hipGraph launch)
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_key[4] = {-1, -1, -1, -1};  // precision bytes, nrhs, criterion, iterations
    const void *graph_ptrs[3] = {nullptr, nullptr, nullptr};
    bool autotune = true;
    bool tuned = false;
    // FFT variant per precision ([0] FP32, [1] FP64): xy-plane kernels (1) or
    // separate x and y passes (0) where both exist, and the z-pass tile (0:
    // default columns per workgroup, 1: the alternative); fixed by the option
    // fft_variant or timed at the first solve of a precision
    int fft_plane[2] = {1, 1};
    int fft_ztile[2] = {0, 0};
    bool fft_tuned[2] = {false, false};
    // cached voxel matrices: option (-1 autotuned, 0 never, 1 always), the
    // tables of each precision (built for the current moduli) and whether the
    // CG iterations of that precision use them
    int vm_mode = -1;
    double *vm64 = nullptr;
    float *vm32 = nullptr;
    bool vm_valid = false;     // tables match the current moduli
    bool vm_on[2] = {false, false};   // [0] FP32, [1] FP64
    bool vm_tuned[2] = {false, false};
    bool last_op_vm = false;   // the last operator launch used the cached matrices
    // profiling hook: events recorded before (id -1) and after (kernel id) every launch
    bool prof_on = false;
    std::vector<hipEvent_t> prof_pool;   // reusable events
    std::vector<int> prof_ids;           // id of the i-th recorded event
    size_t prof_used = 0;
};
