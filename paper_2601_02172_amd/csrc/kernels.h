// Kernel launchers of the X-FFT GPU library (internal).
#pragma once

#include "common.h"

namespace xfft {

SlotLayout slot_layout(const Geometry &g);
// regular-voxel operator depth (planes per block); kz in {4, 8, 16}
void set_depth(SlotLayout &L, const Geometry &g, int kz);
int green_slots(const Geometry &g);
// false when a line FFT of the grid would exceed what the generic passes handle
bool fft_sizes_ok(int n0, int n1, int n2);
// z-pass workgroups per right-hand side in the problem's FFT variant
template <typename T> int green_blocks(const xfft_problem *p);
// the FFT variants a grid has in precision T: bit 0 set when the xy-plane
// kernels and separate passes both exist, bit 1 when the z pass has two tiles
template <typename T> int fft_variants(const Geometry &g);

// Operator r(x) = A x + (macro-strain term) on up to nrhs right-hand sides.
// x/xe may be null (zero input).  sign multiplies the outputs.  When flags is
// non-null a right-hand side r is skipped unless flags[r].active[parity].
// Partial sums: dot (y . x) and the stress integral go to the operator slots.
template <typename T>
void launch_operator(xfft_problem *p, Work<T> &w, const Tables<T> &tb, const T *x, const T *xe, T *y, T *ye,
                     bool use_ebar, T sign, int nrhs, const Flags *flags, int parity, double *vstress,
                     hipStream_t s, bool stress = true);

// The same with explicit work space: macro strains ebar[nrhs][6] (device),
// corner-force buffer cutbuf (48 cut_rows(nirr) values per right-hand side)
// and partial-sum slots partial (nslots NPART doubles per right-hand side).
// allow_vm: the cached voxel matrices may replace the moment form (CG
// iterations); their partial sums then go to the slots after the enriched ones.
template <typename T>
void launch_operator_ws(xfft_problem *p, const Tables<T> &tb, const T *x, const T *xe, T *y, T *ye,
                        const double *ebar, bool use_ebar, T sign, int nrhs, const Flags *flags, int parity,
                        double *vstress, hipStream_t s, bool stress, T *cutbuf, double *partial, bool allow_vm);

// Cached voxel matrices (0; -2 allocation failed; -3 device error) and their release.
int build_voxel_matrices(xfft_problem *p, bool fp32, bool fp64);
void free_voxel_matrices(xfft_problem *p);

// Allocation-free entry point: looks up this device's static scratch area
// (once per device; call with the device current).  0 or XFFT_EDEVICE.
int static_scratch_init(int device);

// Green operator passes.  mode_x_fwd: the residual update f -= alpha z is fused
// when z is non-null.  The z pass writes the Parseval partials.  The enriched
// residual update of launch_enr_update (mode enr_mode, output enr_out) follows
// at the same point: as extra workgroups of the compile-time z pass, else as a
// kernel of its own.
template <typename T>
void launch_green_forward(xfft_problem *p, Work<T> &w, const Tables<T> &tb, T *f, const T *z, int nrhs,
                          const Flags *flags, int parity, hipStream_t s, int enr_mode, T *enr_out);

// mode 0: out = P^-1 f (FE part) written to `out`; mode 1: CG update
// (u += alpha d_old, d = y + beta d_old); mode 2: d = y.  The enriched update
// of launch_enr_final (enr_mode 1 or 2; 0: none) runs inside the xy-plane
// kernels when they are used, else as a kernel of its own.
template <typename T>
void launch_green_inverse(xfft_problem *p, Work<T> &w, const Tables<T> &tb, int mode, T *out, int nrhs,
                          const Flags *flags, int parity, hipStream_t s, int enr_mode);

// Enriched block: mode 0 residual partial only (out = f~ written when out non-null);
// mode 1: f~ -= alpha z~ then partial.
template <typename T>
void launch_enr_update(xfft_problem *p, Work<T> &w, int mode, T *out, int nrhs, const Flags *flags, int parity,
                       hipStream_t s);
// mode 1: u~ += alpha d~, d~ = f~ + beta d~;  mode 2: d~ = f~
template <typename T>
void launch_enr_final(xfft_problem *p, Work<T> &w, int mode, int nrhs, const Flags *flags, int parity,
                      hipStream_t s);
// kernel arguments of the two enriched updates (enriched.h)
template <typename T> struct EnrUpd;
template <typename T> struct EnrFin;
template <typename T> EnrUpd<T> enr_update_args(xfft_problem *p, Work<T> &w, int mode, T *out);
template <typename T> EnrFin<T> enr_final_args(xfft_problem *p, Work<T> &w, int mode);

// Scalar recurrences (one block per right-hand side).
enum ScalarOp { SC_INIT_SIGMA = 0, SC_INIT_RES = 1, SC_ALPHA = 2, SC_BETA = 3, SC_SUM_ONLY = 4, SC_SUM_GREEN = 5 };
// fp64 selects the Green-pass slot count of the FP64 (true) or FP32 (false) kernels.
void launch_scalars(xfft_problem *p, int op, int crit, int nrhs, int parity, double *sum_out, hipStream_t s,
                    bool fp64);

// Vector helpers for iterative refinement.
void launch_round_to_float(xfft_problem *p, int nrhs, hipStream_t s);       // w32.f/fe <- w64.f/fe, w32.u/ue <- 0
void launch_accumulate_correction(xfft_problem *p, int nrhs, hipStream_t s); // w64.u/ue += w32.u/ue

// dC[nphase][2][6][6] from the stored unit-load solutions (0 ok, -1 too many
// phases, -2 allocation, -3 device error).
int grad_tables(xfft_problem *p, double *dC_host);

// Setup.
int run_setup(xfft_problem *p, const double *L_dev_raw);
int compute_tables(xfft_problem *p);

}  // namespace xfft
