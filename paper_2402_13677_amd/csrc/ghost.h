// Ghost velocities of Eq. ghost_velocity (Sec. 2.3): the face rule shared by
// the projection (cut faces) and the narrow-band call (every band face).
//
// With n the unit normal from vapour into liquid and [1/rho] =
// 1/rho_l - 1/rho_v, the field of the phase that does not own a face takes
//   u_vap = u_liq + mdot [1/rho] n_a   (a liquid face),
//   u_liq = u_vap - mdot [1/rho] n_a   (a vapour face),
// so u_vap - u_liq = mdot [1/rho] n_a on every face that gets a ghost.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebit_internal.h"

namespace ebit {

// The cut face fi of axis a between cells lo (below) and hi (above), theta t
// from the lower centre: the face belongs to the lower cell's phase if
// t > 1/2, to the upper's if t < 1/2, to the liquid at 1/2; mdot and n_a are
// those of the cell holding the crossing (t <= 1/2: the lower one) or, if
// that cell carries no facet, of the other.
__device__ inline void cut_face_ghost(const Dims& d, const uint8_t* flags, const double* nF, const double* mdot,
                                      double jump, int a, long long lo, long long hi, double t, long long fi,
                                      double* ul, double* uv) {
  const int col_lo = (flags[lo] & F_LIQ) ? 1 : 0, col_hi = (flags[hi] & F_LIQ) ? 1 : 0;
  const int kf = (t > 0.5) ? col_lo : ((t < 0.5) ? col_hi : 1);
  long long hold = (t <= 0.5) ? lo : hi;
  if (!(flags[hold] & F_IF)) hold = (hold == lo) ? hi : lo;
  const double jmp = mdot[hold] * jump * nF[a * d.N + hold];
  if (kf == 1)
    uv[fi] = ul[fi] + jmp;
  else
    ul[fi] = uv[fi] - jmp;
}

}  // namespace ebit

// Eq. ghost_velocity on every face of the narrow band (both cells band
// cells), from a mass flux already carried to the band: cut faces as in the
// projection; an uncut face belongs to the common phase of its cells and
// takes the means of the two cells' mass flux and unit band normals.
// bytes: 2 N bytes of scratch; nb: dim arrays of N doubles of scratch (the
// band cells' unit normals); counter: one int of scratch.
extern "C" hipError_t ebit_launch_ghost_band(const ebit::Dims* d, double jump, const uint8_t* flags,
                                             const double* const th[3], const double* nF, const double* mdot,
                                             double* const ul[3], double* const uv[3], uint8_t* bytes,
                                             double* const nb[3], int* counter, hipStream_t st);
