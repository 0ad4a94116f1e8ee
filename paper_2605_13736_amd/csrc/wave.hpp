#pragma once
// Wave-wide (64-lane) reductions on data-parallel-primitive (DPP) lane moves.
//
// A lane move through DPP is a VALU operand modifier: it costs one VALU
// instruction and no LDS round trip, where a __shfl_xor step is a
// ds_bpermute through the LDS crossbar with its full latency.  A reduction
// combines within quads (xor 1, xor 2), then rotates within each row of 16
// lanes by 4 and by 8, after which every lane of a row holds the row's
// result; readlane of lanes 0, 16, 32 and 48 then combines the four rows in
// the same order in every lane.  All 64 lanes must be active.
#include <hip/hip_runtime.h>

namespace mds {
namespace wave {

constexpr int kXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kRor4 = 0x124; // row_ror:4
constexpr int kRor8 = 0x128; // row_ror:8

template <int C>
__device__ inline int dpp(int v) {
  return __builtin_amdgcn_update_dpp(v, v, C, 0xf, 0xf, false);
}
template <int C>
__device__ inline double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp<C>((int)b), hi = dpp<C>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// larger magnitude, then smaller position (a total order: every lane ends
// with the same pair whatever the combination order)
__device__ inline void amax2(double &v, int &i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}
__device__ inline void amax3(double &v, int &i, int &s, double v2, int i2, int s2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
    s = s2;
  }
}

template <int C>
__device__ inline void amax_step(double &v, int &i) {
  const double v2 = dpp<C>(v);
  const int i2 = dpp<C>(i);
  amax2(v, i, v2, i2);
}
template <int C>
__device__ inline void amax_step(double &v, int &i, int &s) {
  const double v2 = dpp<C>(v);
  const int i2 = dpp<C>(i), s2 = dpp<C>(s);
  amax3(v, i, s, v2, i2, s2);
}

// arg-max of (v, i) over the 16 lanes of each row: every lane of the row
__device__ inline void row_amax(double &v, int &i) {
  amax_step<kXor1>(v, i);
  amax_step<kXor2>(v, i);
  amax_step<kRor4>(v, i);
  amax_step<kRor8>(v, i);
}
__device__ inline void row_amax(double &v, int &i, int &s) {
  amax_step<kXor1>(v, i, s);
  amax_step<kXor2>(v, i, s);
  amax_step<kRor4>(v, i, s);
  amax_step<kRor8>(v, i, s);
}

// arg-max over the wave, result in every lane (wave-uniform)
__device__ inline void amax(double &v, int &i) {
  row_amax(v, i);
  double r = lane_read(v, 0);
  int ri = lane_read(i, 0);
  amax2(r, ri, lane_read(v, 16), lane_read(i, 16));
  amax2(r, ri, lane_read(v, 32), lane_read(i, 32));
  amax2(r, ri, lane_read(v, 48), lane_read(i, 48));
  v = r;
  i = ri;
}
__device__ inline void amax(double &v, int &i, int &s) {
  row_amax(v, i, s);
  double r = lane_read(v, 0);
  int ri = lane_read(i, 0), rs = lane_read(s, 0);
  amax3(r, ri, rs, lane_read(v, 16), lane_read(i, 16), lane_read(s, 16));
  amax3(r, ri, rs, lane_read(v, 32), lane_read(i, 32), lane_read(s, 32));
  amax3(r, ri, rs, lane_read(v, 48), lane_read(i, 48), lane_read(s, 48));
  v = r;
  i = ri;
  s = rs;
}

// maximum over the wave (fmax: a NaN operand is ignored), every lane
__device__ inline double max(double v) {
  v = fmax(v, dpp<kXor1>(v));
  v = fmax(v, dpp<kXor2>(v));
  v = fmax(v, dpp<kRor4>(v));
  v = fmax(v, dpp<kRor8>(v));
  double r = fmax(lane_read(v, 0), lane_read(v, 16));
  return fmax(r, fmax(lane_read(v, 32), lane_read(v, 48)));
}

// sum over the wave, every lane (association: quads, rows, then rows 0..3)
__device__ inline double sum(double v) {
  v = v + dpp<kXor1>(v);
  v = v + dpp<kXor2>(v);
  v = v + dpp<kRor4>(v);
  v = v + dpp<kRor8>(v);
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

}  // namespace wave
}  // namespace mds
