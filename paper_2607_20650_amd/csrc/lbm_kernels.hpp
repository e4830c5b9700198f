// lbm_kernels.hpp -- host-callable launchers of the device kernels.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

// One lattice update.  Two-lattice schemes read src and write dst; one-lattice
// schemes update dst in place and read / write the edge buffers ein / eout.
hipError_t launch_update(int scheme, int layout, int prec, const KParams& p, int block, const void* src, void* dst,
                         const void* ein, void* eout, hipStream_t s);

// One AA update in place on lat.  parity 0: even update (local; push state
// -> swap state; also writes the outlet side buffer obuf, 3 values per row,
// when the x axis is inflow/outflow).  parity 1: odd update (pairwise
// exchange; swap state -> push state; reads obuf).
hipError_t launch_aa(int layout, int prec, const KParams& p, int parity, void* lat, void* obuf, hipStream_t s);

// The AA outlet side buffer from a swap-state lattice (after a state load at
// odd parity): obuf[3 y + k] = f*_{3k} of the outlet node of row y.
hipError_t launch_aa_outlet_fill(int layout, int prec, const KParams& p, const void* lat, void* obuf, hipStream_t s);

// Neumann inlet: rin[y] = rho - 1 of the node (1, y) in the shifted
// post-collision values f [9][ny][nx] (FP32, device), 0 where it is not updated.
hipError_t launch_inlet_density_fill(const KParams& p, const float* f, float* rin, hipStream_t s);

// Block size the occupancy query picks for the linear (LPTL) kernel.
int lptl_block_size(int layout, int prec);

// Node types from user flags (device arrays): flags [ny][nx] -> types [ny][px].
hipError_t launch_types(const Geometry& g, const uint8_t* flags, uint8_t* types, hipStream_t s);
// Per-node link words (KParams::links) from the node types.
hipError_t launch_links(const Geometry& g, const uint8_t* types, uint32_t* links, hipStream_t s);

// Initial state of a scheme's state kind into lat (every slot of every node).
hipError_t launch_init(int state, int layout, int prec, const KParams& p, void* lat, hipStream_t s);

// Load a canonical post-collision state f [9][ny][nx] (FP32, device).  For
// the push state, tmp (a second lattice) receives the pull form first.
hipError_t launch_set_state(int state, int layout, int prec, const KParams& p, const float* f, void* lat, void* tmp,
                            hipStream_t s);

// Fill one parity of the one-lattice edge buffers from a pull / swap lattice.
hipError_t launch_edge_fill(int state, int layout, int prec, const KParams& p, const void* lat, void* edge,
                            hipStream_t s);

// Canonical incoming populations [9][ny][nx] (FP32, device).
hipError_t launch_get_populations(int state, int layout, int prec, const KParams& p, const void* lat, float* f,
                                  hipStream_t s);

// rho [ny][nx] and u [2][ny][nx] (FP32, device); either may be null.
hipError_t launch_macros(int state, int layout, int prec, const KParams& p, const void* lat, float* rho, float* u,
                         hipStream_t s);

// FP64 diagnostics: out[0..4] = mass, jx, jy, residual numerator^2,
// denominator^2; u_prev (2 doubles per node, dense [ny][nx][2]; may be null:
// no residual terms) is read when have_prev and overwritten with the current
// velocity.  partials holds diag_partials() doubles.
int diag_partials();
hipError_t launch_diag(int state, int layout, int prec, const KParams& p, const void* lat, double* u_prev,
                       int have_prev, double* partials, double* out, hipStream_t s);
// out[0..3] = mass, jx, jy, residual (-1 without have_prev) from the five
// sums launch_diag wrote to `sums` (device).
hipError_t launch_diag_result(const double* sums, int have_prev, double* out, hipStream_t s);

} // namespace lbm

namespace lbm {
// Bandwidth probe: mode 0 copy src -> dst, 1 read src (dst: 4-byte sink),
// 2 write dst; bytes a multiple of 16, pointers 16-byte aligned.
hipError_t launch_probe(int mode, void* dst, const void* src, int64_t bytes, hipStream_t s);
} // namespace lbm
