// lbm_launch.hpp -- host-side launch interface between the C-ABI layer and
// the step kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"
#include "lbm_fstar.hpp"

namespace lbm {

// candidate of the Ehrenfests' ranking: site and its FP64 Delta S
struct Cand {
  uint32_t site;
  uint32_t pad;
  double ds;
};

// device-side statistics written by the selection kernel
struct DevStats {
  unsigned long long n_above, n_sel, n_invalid, total_sel;
  unsigned long long n_screened;  // entries of the candidate array (screened sites)
  double kth, max;
  double sums[4];
};

// device counters (uint32 each)
enum : int {
  C_SCREEN = 0,    // sites that passed the FP32 screen this step
  C_CAND = 1,      // sites with FP64 Delta S > delta this step
  C_INVALID = 2,   // candidates with Delta S = +inf
  C_NONFINITE = 3, // sticky halt: 0, or 1 + (buffer written by the first step
                   // that met non-finite values) + 2 (if that step read the
                   // canonical layout); every later step kernel returns at once
  C_NSEL0 = 4,     // sites selected by k_partition (above the bin b*)
  C_SETBAD = 5,    // set_populations met a non-finite value
  C_BADSTEP = 6,   // number of that first non-finite step (1 = the first step)
  C_BSTAR = 7,     // histogram bin holding the k-th largest key
  C_R = 8,         // keys still to take from bin b*
  C_NBND = 9,      // candidates in bin b* (boundary list)
  C_STEP0 = 10,    // C_STEP0 + d: number of the last step that wrote buffer d
  C_COUNT = 16
};

constexpr int HIST_BITS = 15;
constexpr int HIST_BINS = 1 << HIST_BITS;
// coarse histogram behind the fine one: coarse bin c counts fine bins
// [256 c, 256 c + 256), so that the bin of the k-th key is found from 128 +
// 256 coalesced counts
constexpr int HIST_COARSE = HIST_BINS / 256;
constexpr int HIST_WORDS = HIST_BINS + HIST_COARSE;
// workgroups of the partition kernel (one per-workgroup max / min each)
constexpr int PART_BLOCKS = 1024;
constexpr int STEP_TX = 256;  // sites per step-kernel block (one row segment)
// workgroups of the conservation sums (per-workgroup FP64 partials, added in
// fixed order): enough sites in flight to stream the state from HBM
constexpr int SUM_BLOCKS = 8192;

struct StepArgs {
  const void* A;   // state read this step
  void* B;         // state written this step
  int dst;         // index (0 or 1) of the buffer B
  Geom g;
  uint32_t* ctr;
  uint32_t* screen;  // [N]: the screened sites of the step (C_SCREEN of them)
  unsigned long long* part;  // [2][PART_BLOCKS]: per-workgroup max of all candidates
                             // and min of the selected ones (Delta S bits)
  Cand* cand;
  Cand* bnd;
  uint32_t* hist;
  uint32_t* sel;
  double* sel_ds;
  DevStats* st;
  double* partials;  // [SUM_BLOCKS][4] FP64 block partials of the conservation sums
  double* Mbuf;      // f*_M only: moments [4][N] of the current step
  const double* mu;  // f*_M only: multipliers [4][N] of the current step
  float thr_a, thr_b;  // FP32 screen threshold: thr_a - thr_b * sqrt(rho)
  int64_t ntx, nblocks;
  int prec, Q, qe;
  int coll;  // 0 LBGK, 1 ELBM
  int one_wg;  // ranking and selection by one workgroup (k_select_one)
  // f*_M time step: workgroups of k_fstep for the canonical [0] and pulled
  // [1] layouts, the number the device holds at once (0: FSTAR_MAX_BLOCKS)
  int fgrid[2];
  // monitoring point: site index (-1: none), ring [3][probe_cap] of
  // (rho, u1, u2) of f(x, t), and the device count of recorded samples
  int64_t probe;
  double* probe_buf;
  int64_t probe_cap;
  unsigned long long* probe_n;
};

// launch one step's kernels (fused step, rank, select, reset) on stream s;
// ev0/ev1 (optional) bracket the fused step kernel
hipError_t launch_step(const StepArgs& a, bool pull, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

hipError_t launch_init(const StepArgs& a, const double* rho0, const double* u0, const double* twoE0,
                       hipStream_t s);
// f*_M: moments of the current pre-collision state into a.Mbuf (solid sites
// get the isothermal rest moments so that the solver has a feasible input)
hipError_t launch_moments_M(const StepArgs& a, bool pull, hipStream_t s);
// f*_M time step without a network start: the statistics clear, the pull,
// moments, Newton solve (start: START_REST, START_CLOSED or START_PREV),
// screen and collision of every fluid site in one kernel (bracketed by
// ev0 / ev1 when given), the damped fallback with the collision of its
// sites, then ranking and selection
hipError_t launch_fstep(const StepArgs& a, const FstarArgs& fa, int start, bool pull, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1);
// workgroups of the f*_M step kernel of this precision, start, layout and
// collision that the device holds at once (occupancy x compute units), or 0
int fstep_resident(int prec, int start, bool pull, bool elbm);
// f*_M initial state: moments of the initial fields into a.Mbuf, and (after
// the solve) f = f*(mu) into the state buffer a.B
hipError_t launch_init_M_moments(const StepArgs& a, const double* rho0, const double* u0, const double* twoE0,
                                 hipStream_t s);
hipError_t launch_init_M_pops(const StepArgs& a, hipStream_t s);
hipError_t launch_get(const StepArgs& a, bool pull, void* out, hipStream_t s);
hipError_t launch_set(const StepArgs& a, const void* in, hipStream_t s);
hipError_t launch_moments(const StepArgs& a, bool pull, double* rho, double* rhou, double* e2,
                          hipStream_t s);
// power spectrum |DFT|^2 of a real signal x[n] at bins 0..n/2 (FP64), and
// the bin k >= 1 of largest power (lowest k on ties) into *peak (device)
hipError_t launch_dft_power(const double* x, int64_t n, double* power, int64_t* peak, hipStream_t s);
// FP64 conservation sums of the current pre-collision state into st->sums
hipError_t launch_sums(const StepArgs& a, bool pull, hipStream_t s);
hipError_t launch_clear(const StepArgs& a, hipStream_t s);

}  // namespace lbm
