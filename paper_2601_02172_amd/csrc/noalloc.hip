// Allocation-free operator application (xfft_apply_operator_noalloc).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops): the work space of the operator kernels -- the
// per-workgroup partial sums and the corner-force buffer of the irregular
// voxels -- lives in a file-scope device array of fixed size instead of
// buffers of the problem.  Every GPU the library runs on holds its own copy of
// the array until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for that device.
#include "../../include/xfft.h"
#include "kernels.h"

#include <mutex>

namespace xfft {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per device
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_addr[MAX_DEVICES] = {};

// Sum of the operator's partial-sum slots (regular-voxel blocks, then the
// irregular-voxel and enriched-gather blocks) in the order of the scalar
// recurrences, converted to the Mandel average stress of the cell.
__global__ __launch_bounds__(256) void k_avg_stress(const double *partial, int s0, int n, int s1, int n1,
                                                     double volume, double *avg) {
    __shared__ double red[4 * 7];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] += partial[(int64_t)(s0 + i) * NPART + q];
    }
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] += partial[(int64_t)(s1 + i) * NPART + q];
    }
    block_sum<7>(v, red);
    if (threadIdx.x == 0) {
        const double r2 = 1.41421356237309504880;
        avg[0] = v[1] / volume; avg[1] = v[2] / volume; avg[2] = v[3] / volume;
        avg[3] = r2 * v[4] / volume; avg[4] = r2 * v[5] / volume; avg[5] = r2 * v[6] / volume;
    }
}

}  // namespace

int static_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return XFFT_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_addr[device]) return XFFT_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return XFFT_EDEVICE;
    g_addr[device] = ptr;
    return XFFT_OK;
}

}  // namespace xfft

using namespace xfft;

extern "C" int xfft_apply_operator_noalloc(xfft_problem *p, const double *x_dev, const double *macro_strain_dev,
                                           double *y_dev, double *avg_stress_dev, void *stream) {
    if (!p || !x_dev || !y_dev) return XFFT_EINVAL;
    if (p->prof_on) return XFFT_EINVAL;          // the profiling hook creates events
    if (p->device < 0 || p->device >= MAX_DEVICES) return XFFT_EDEVICE;
    const Geometry &g = p->g;
    const size_t part_bytes = sizeof(double) * NPART * (size_t)p->nslots;
    const size_t part_off = 0;
    const size_t cut_off = (part_bytes + 255) & ~(size_t)255;
    const size_t cut_bytes = sizeof(double) * 48 * (size_t)cut_rows(g.nirr);
    if (cut_off + cut_bytes > SCRATCH_BYTES) return XFFT_EINVAL;
    if (hipSetDevice(p->device) != hipSuccess) return XFFT_EDEVICE;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        base = static_cast<unsigned char *>(g_addr[p->device]);
    }
    if (!base) return XFFT_EDEVICE;              // set up by xfft_setup on this device
    double *partial = reinterpret_cast<double *>(base + part_off);
    double *cutbuf = reinterpret_cast<double *>(base + cut_off);
    hipStream_t s = stream ? (hipStream_t)stream : p->stream;
    // every workgroup writes its own partial-sum slot and every irregular voxel
    // its corner-force rows before they are read, so nothing needs clearing
    launch_operator_ws<double>(p, p->t64, x_dev, x_dev + 3 * g.N, y_dev, y_dev + 3 * g.N, macro_strain_dev,
                               macro_strain_dev != nullptr, 1.0, 1, nullptr, 0, nullptr, s, avg_stress_dev != nullptr,
                               cutbuf, partial, false);
    const SlotLayout &L = p->slots;
    if (avg_stress_dev)
        k_avg_stress<<<1, 256, 0, s>>>(partial, L.fe0, L.fe_n, L.cut0, L.cut_n + L.enr_n, (double)g.N,
                                       avg_stress_dev);
    if (hipGetLastError() != hipSuccess) return XFFT_EDEVICE;
    return XFFT_OK;
}
