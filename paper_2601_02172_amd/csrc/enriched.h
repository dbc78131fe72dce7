// Vector updates of the enriched block of the CG (the preconditioner is the
// identity on the scaled enriched dofs, eq. scaledPreconditioner).  Device
// functions, so that the updates run either as kernels of their own or as
// extra workgroups of the Green passes that sit at the same point of the
// iteration.
#pragma once

#include "common.h"

namespace xfft {

constexpr int ENR_BLOCK = 512;   // enriched nodes per residual-update workgroup (one partial slot)

// Residual update: mode 0 partial only (out = f~ when out is non-null);
// mode 1: f~ -= alpha z~ first.  Partial: f~ . f~ (= f~ . P^-1 f~).
template <typename T> struct EnrUpd {
    int64_t nX = 0;
    int mode = 0;
    T *fe = nullptr;
    const T *ze = nullptr;
    T *out = nullptr;
    int nblk = 0;         // workgroups (= partial slots) per load, 0: not fused
    int slot0 = 0;
};

// Workgroup b of load r (blockDim.x == ENR_BLOCK); red holds ENR_BLOCK / 64 doubles.
template <typename T>
__device__ __forceinline__ void enr_update_block(const EnrUpd<T> &E, const Scalars *scal, double *partial,
                                                 int nslots, int r, int b, double *red) {
    const int64_t nX = E.nX;
    const int64_t j = (int64_t)b * ENR_BLOCK + threadIdx.x;
    double acc[1] = {0.0};
    if (j < nX) {
        const T alpha = (T)scal[r].alpha;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t o = (int64_t)r * 3 * nX + c * nX + j;
            T v = E.fe[o];
            if (E.mode == 1) {
                v -= alpha * E.ze[o];
                E.fe[o] = v;
            }
            if (E.out) E.out[o] = v;
            acc[0] += (double)v * (double)v;
        }
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) {
        double *P = partial + ((int64_t)r * nslots + E.slot0 + b) * NPART;
        P[0] = acc[0];
#pragma unroll
        for (int q = 1; q < 7; ++q) P[q] = 0.0;
    }
}

// Direction update: mode 1: u~ += alpha d~, d~ = f~ + beta d~;  mode 2: d~ = f~.
template <typename T> struct EnrFin {
    int64_t nX = 0;
    int mode = 0;         // 0: not fused
    T *ue = nullptr, *de = nullptr;
    const T *fe = nullptr;
};

// Nodes j0, j0 + stride, ... of load r.
template <typename T>
__device__ __forceinline__ void enr_final_rows(const EnrFin<T> &E, const Scalars *scal, int r, int64_t j0,
                                               int64_t stride) {
    const int64_t nX = E.nX;
    const T alpha = (T)scal[r].alpha, beta = (T)scal[r].beta;
    for (int64_t j = j0; j < nX; j += stride) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t o = (int64_t)r * 3 * nX + c * nX + j;
            if (E.mode == 1) {
                const T d = E.de[o];
                E.ue[o] += alpha * d;
                E.de[o] = E.fe[o] + beta * d;
            } else {
                E.de[o] = E.fe[o];
            }
        }
    }
}

}  // namespace xfft
