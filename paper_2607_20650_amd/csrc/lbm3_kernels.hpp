// lbm3_kernels.hpp -- host-callable launchers of the D3Q19 kernels.
#pragma once

#include "lbm3.hpp"

namespace lbm {

// Node types from user flags (device arrays): flags [nz][ny][nx] -> types [nz][ny][px].
hipError_t launch3_types(const Geometry3& g, const uint8_t* flags, uint8_t* types, hipStream_t s);

// Initial state of a state kind into lat.
hipError_t launch3_init(int state, int layout, int prec, const KParams3& p, void* lat, hipStream_t s);

// Load shifted post-collision values f [19][nz][ny][nx] (FP32, device); the
// push form is built through tmp (a second lattice).
hipError_t launch3_set_state(int state, int layout, int prec, const KParams3& p, const float* f, void* lat, void* tmp,
                             hipStream_t s);

// One update.  PULL: src -> dst.  AA: in place on dst, parity 0 even, 1 odd,
// with the outlet side buffer obuf (5 values per (y, z) row; inflow/outflow x
// axis only).
hipError_t launch3_update(int scheme, int layout, int prec, const KParams3& p, int parity, const void* src, void* dst,
                          void* obuf, hipStream_t s);

// The AA outlet side buffer from a swap-form lattice.
hipError_t launch3_aa_outlet_fill(int layout, int prec, const KParams3& p, const void* lat, void* obuf, hipStream_t s);

// Incoming populations [19][nz][ny][nx] and rho [nz][ny][nx], u [3][nz][ny][nx] (FP32, device).
hipError_t launch3_get_populations(int state, int layout, int prec, const KParams3& p, const void* lat, float* f,
                                   hipStream_t s);
hipError_t launch3_macros(int state, int layout, int prec, const KParams3& p, const void* lat, float* rho, float* u,
                          hipStream_t s);

// FP64 diagnostics: out[0..5] = mass, jx, jy, jz, sum |u - u_prev|^2,
// sum |u|^2; u_prev (3 doubles per padded node) read when have_prev and
// overwritten.  partials holds diag3_partials() doubles.
int diag3_partials();
hipError_t launch3_diag(int state, int layout, int prec, const KParams3& p, const void* lat, double* u_prev,
                        int have_prev, double* partials, double* out, hipStream_t s);

} // namespace lbm
