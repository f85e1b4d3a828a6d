// Host-side interface of the HIP kernels (plain pointers, no torch types).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace islbm {

// Everything a kernel needs about one context, in double precision; the
// launchers convert to the arithmetic type of the storage.
struct DevState {
  int dim;         // 2 or 3
  int storage;     // islbm_storage
  int n[3];        // fluid nodes per axis (n[2] = 1 in 2-D)
  int pitch;       // row pitch in elements (>= n[0])
  long long plane; // elements per population (pitch x n[1] x n[2])
  long long ps;    // elements between the rows of two populations of a (z, y) row
  long long rsf;   // elements between consecutive rows of one f population
  long long rsg;   // elements between consecutive rows of one g population
  // relaxation and physics, lattice units
  double s_e, s_eps, s_q, s_nu, s_pi, s_m, q_j, q_e, q_nu, aT;
  double gbeta, T0, omega, Thot, Tcold;
  double inv_uf, inv_dT;
  int collide;     // 0 => collision is the identity
  int uniform;     // 1 => every interpolation weight is one-hot (uniform mesh)
  int large;       // read + write population buffers: 0 fit the last-level cache,
                   // 1 exceed it, 2 exceed 1 GB
  // per-axis interpolation weights: axis a holds [2][n[a]][4] of float or
  // double (first block: lattice direction +1, second: -1); wall links are 0
  const void* wtab[3];
  // reduction coefficients (double): vol[a][n[a]] (V/extent), mw[a][n[a]]
  // (V/Delta), then chot, ccold, cmv, cmd over n[0]
  const double* red;
  long long red_vol[3], red_mw[3], red_chot, red_ccold, red_cmv, red_cmd;
  // stochastic rounding of 2-byte storage: two device step counters; a step
  // launch reads rctr[rpar] and writes rctr[rpar ^ 1] (rpar = buffer parity)
  unsigned int* rctr;
  int rpar;
};

constexpr int kRedSlots = 13;  // 8 sums, 3 maxima, 1 non-finite count, 1 sum (|u*|^2)

int step_blocks(const DevState& s);
hipError_t launch_step(const DevState& s, const void* fin, const void* gin, void* fout,
                       void* gout, bool reduce, double* partials, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t st);
// One population between a dense FP64 node array (x fastest) and its rows in
// a population buffer: dst / src point at the population's first row (the
// buffer plus pop * ps elements); flow = 1 for f (weights subtracted / added
// back), 0 for g.
hipError_t launch_convert_in(const DevState& s, const double* src, void* dst, int pop, int flow,
                             hipStream_t st);
hipError_t launch_convert_out(const DevState& s, const void* src, double* dst, int pop, int flow,
                              hipStream_t st);
hipError_t launch_collide_only(const DevState& s, const void* fin, const void* gin, void* fout,
                               void* gout, hipStream_t st);
hipError_t launch_init_eq(const DevState& s, const double* ux, const double* uy,
                          const double* uz, const double* T, void* fout, void* gout,
                          hipStream_t st);
hipError_t launch_fields(const DevState& s, const void* f, const void* g, double* rho, double* ux,
                         double* uy, double* uz, double* T, hipStream_t st);
int reduce_state_blocks(const DevState& s);
hipError_t launch_reduce_state(const DevState& s, const void* f, const void* g, double* partials,
                               hipStream_t st);
hipError_t launch_finish(const double* partials, int nblocks, double* out, hipStream_t st);
hipError_t launch_steady_change(const DevState& s, const void* f, const void* g, double* snap, int first,
                                double* partials, hipStream_t st);

}  // namespace islbm
