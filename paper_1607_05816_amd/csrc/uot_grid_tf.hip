// Tile-factored separable grid pass of libuot on gfx950 MFMA (the dominant
// kernel of grid solves), with its launchers.
#include <algorithm>
#include <cstdlib>

#include "uot_device.h"
#include "uot_epilogue.h"
#include "uot_launch.h"

// ---------------------------------------------------------------------------
// Tile-factored separable pass on FP32 MFMA.  For output tile I and tap tile J
// of 16 cells each (centres cI, cJ, offsets e = i - cI, f = j - cJ, D = cI -
// cJ, all in cells) the 1-D kernel g(i - j) = -c (i - j)^2 (c = h^2 log2(e) /
// eps) splits exactly as
//   g = [-c e (e + 2D)] + [-c f (f - 2D)] - c D^2 + 2 c e f,
// so  sum_j 2^{g + w_j} = 2^{-c e (e+2D) - c D^2 + m} * sum_j Khat[e][f] E_j,
//   Khat[e][f] = 2^{2 c e f}  (one 16 x 16 matrix, |2 c e f| <= 2 c 7.5^2),
//   E_j = 2^{w_j - c f (f - 2D) - m},  m = max_j (w_j - c f (f - 2D)),
// and the inner sums of 16 lines at once are one 16x16x16 FP32 MFMA product.
// The J tiles of an output are combined by an online log-sum-exp.  Exact up
// to FP32 rounding; exp2 count per output: 16/16 (E) + 2 per J tile instead of
// 16 per J tile.  Requires n % 16 == 0.
// HALF: Khat and E in FP16, one v_mfma_f32_16x16x16f16 per J tile (FP32
// accumulation); lane (li, q) then holds taps 4 q .. 4 q + 3 of a tile.  The
// inputs carry FP16 rounding (2^-11 relative), so results are good to ~1e-3;
// Khat stays finite in FP16 while 2 c 7.5^2 <= 15.
//   STRIDED = false: in[a][j], lines a (16 per group);  out[a][i]
//   STRIDED = true : in[a][j][b], lines (a, b), 16 consecutive b per group
// grid = (n/16 output tiles, line groups (y, z)), 4 waves split the J tiles.
// ---------------------------------------------------------------------------
namespace uot {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

template <bool STRIDED, int TPC, bool MULTI, bool HALF>
__global__ __launch_bounds__(kBlock) void k_grid_tf(const float* __restrict__ in, int n, int64_t A, int64_t B,
                                                     int opb, double h, int side, const Ctrl* __restrict__ c,
                                                     EpiArgs<float> ep) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, li = lane & 15;
  const int nt = n / 16;
  // logical block -> (block of opb output tiles, line group of 16 lines)
  const int64_t lid = blockIdx.x;
  const int nob = MULTI ? opb : 1;         // output tiles of this block
  const int tpb = nt / nob;                // output-tile blocks per line group
  const int64_t grp = lid / tpb;
  const int ob = (int)(lid % tpb);
  int64_t a, bb;
  bool valid;
  if (STRIDED) {
    const int64_t gpa = (B + 15) / 16;     // groups per a
    a = grp / gpa;
    bb = (grp % gpa) * 16 + li;
    valid = (a < A) && (bb < B);
  } else {
    a = grp * 16 + li;
    bb = 0;
    valid = a < A;
  }
  const int64_t base = valid ? (STRIDED ? a * (int64_t)n * B + bb : a * (int64_t)n) : 0;
  const int64_t tstride = STRIDED ? B : 1;
  // The wave's tap tiles jt = wv, wv + 4, ... are taken in chunks of TPC
  // (4 TPC loads issued together).  The first chunk and the operands of the
  // first epilogue this wave finishes (outputs i = I0 + 4 q + wv of line li)
  // are loaded before the control block is read, so the latencies overlap.
  // Tap (jt, s) of the lane's line is cell jt * 16 + f(q, s), f = 4 s + q
  // (FP32 operand layout) or 4 q + s (FP16); tiles past the end are read at
  // the last tile (in bounds) and replaced by -inf.  Lanes of
  // a line past the end read line 0 unconditionally: lines never mix (MFMA
  // columns and the max exchanges stay within a line) and their outputs are
  // dropped, while a masked load would serialise the loads.
  auto tapf = [&](int s) -> int { return HALF ? 4 * q + s : 4 * s + q; };
  const float* __restrict__ pl = in + base;
  auto load_chunk = [&](float (&w)[TPC][4], int jc) {
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const int jt = jc + 4 * t;
      const int jtc = jt < nt ? jt : nt - 1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const float x = pl[(int64_t)(jtc * 16 + tapf(s)) * tstride];
        w[t][s] = jt < nt ? x : -__builtin_inff();
      }
    }
  };
  // output element of lane (li, q) in output tile o of the block, row wv
  auto out_elem = [&](int o) -> int64_t {
    const int ie = (ob * nob + o) * 16 + 4 * q + wv;
    return valid ? (STRIDED ? (a * (int64_t)n + ie) * B + bb : a * (int64_t)n + ie) : 0;
  };
  float wv4[TPC][4];
  load_chunk(wv4, wv);
  int64_t eo = out_elem(0);
  EpiIn<float> xin = epi_load<float>(eo, ep);
  // block 0 of a launch that hosts the control step loads the residual
  // partials and control fields now, and finishes the step at the end
  const bool hosting = ep.host_ctl != nullptr && blockIdx.x == 0;
  const int par = par_of(side);
  CtrlSnap hsnap{};
  float hm = -__builtin_inff(), hden = 0.f, hnum = 0.f, hdu = 0.f;
  if (hosting) {
    hsnap = ctrl_snap(ep.host_ctl, par);
    ctl_load(ep.host_parts, ep.host_nparts, hm, hden, hnum, hdu);
  }
  // keep those loads ahead of the branch (otherwise they may be moved past it)
#pragma unroll
  for (int t = 0; t < TPC; ++t)
#pragma unroll
    for (int s = 0; s < 4; ++s) asm volatile("" ::"v"(wv4[t][s]));
  asm volatile("" ::"v"(xin.ld), "v"(xin.uo), "v"(xin.lp));
  if (skip_side(c, side)) {
    if (hosting && threadIdx.x == 0) control_skip(ep.host_ctl, par);
    return;
  }
  const float cc = float(h * h * kLog2e / eps_of(c, side));
  // Khat as MFMA A operands: entry s of the lane is Khat[i = li][k = f(q, s)]
  float kh[4];
  f16x4_t kh16;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float e = float(li) - 7.5f, f = float(tapf(s)) - 7.5f;
    kh[s] = __builtin_amdgcn_exp2f(2.f * cc * e * f);
    kh16[s] = (_Float16)kh[s];
  }
  // opb > 1 only when one chunk holds all of a wave's tap tiles (the host
  // picks opb so), so the taps stay in registers across the output tiles
  __shared__ float smM[2][4][4][64], smS[2][4][4][64];
  ResAcc<float> ra;
  ra.init();
  for (int o = 0; o < nob; ++o) {
    const int I0 = (ob * nob + o) * 16;
    // epilogue operands of the next output tile, in flight during this one
    const bool more = MULTI && o + 1 < nob;
    const int64_t eo_next = more ? out_elem(o + 1) : eo;
    const EpiIn<float> xin_next = more ? epi_load<float>(eo_next, ep) : xin;
    // running LSE of the 4 outputs i = 4q + r of this lane's line li (D layout)
    float M[4], S[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      M[r] = -__builtin_inff();
      S[r] = 0.f;
    }
    for (int jc = wv; jc < nt; jc += 4 * TPC) {
      if (jc != wv) load_chunk(wv4, jc);
      // the TPC tiles of a chunk are independent until the final merge:
      // column factors and their line maxima first, then the products, so
      // the exchanges and the MFMA chains of different tiles overlap
      float D[TPC], mloc[TPC], beta[TPC][4];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        D[t] = float(I0 - (jc + 4 * t) * 16);
        mloc[t] = -__builtin_inff();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float f = float(tapf(s)) - 7.5f;
          beta[t][s] = wv4[t][s] - cc * (f * (f - 2.f * D[t]));
          mloc[t] = fmaxf(mloc[t], beta[t][s]);
        }
      }
      // max over the 16 taps of the line: the four lane rows q share a line
#pragma unroll
      for (int t = 0; t < TPC; ++t) mloc[t] = max_over_rows(mloc[t]);
      f32x4_t acc[TPC];
      float E[TPC][4];
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const float msh = (mloc[t] == -__builtin_inff()) ? 0.f : mloc[t];
#pragma unroll
        for (int s = 0; s < 4; ++s) E[t][s] = __builtin_amdgcn_exp2f(beta[t][s] - msh);
      }
      if (HALF) {
#pragma unroll
        for (int t = 0; t < TPC; ++t) {
          f16x4_t e16;
#pragma unroll
          for (int s = 0; s < 4; ++s) e16[s] = (_Float16)E[t][s];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(kh16, e16, acc[t], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int t = 0; t < TPC; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(kh[s], E[t][s], acc[t], 0, 0, 0);
      }
      // acc[t][r] = sum_f Khat[e_i][f] E_f for output i = 4 q + r of line li;
      // one rescale of the running sum per chunk
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float e = float(4 * q + r) - 7.5f;
        float al[TPC];
        float mn = M[r];
#pragma unroll
        for (int t = 0; t < TPC; ++t) {
          al[t] = (mloc[t] == -__builtin_inff()) ? -__builtin_inff()
                                                 : (mloc[t] - cc * (e * (e + 2.f * D[t])) - cc * D[t] * D[t]);
          mn = fmaxf(mn, al[t]);
        }
        const float sh = (mn == -__builtin_inff()) ? 0.f : mn;
        float sum = S[r] * __builtin_amdgcn_exp2f(M[r] - sh);
#pragma unroll
        for (int t = 0; t < TPC; ++t) sum += acc[t][r] * __builtin_amdgcn_exp2f(al[t] - sh);
        S[r] = sum;
        M[r] = mn;
      }
    }
    // merge the four waves (each saw a quarter of the J tiles); wave w then
    // finishes output row r = w of every lane.  Two LDS buffers alternate
    // over the output tiles, so one barrier per tile suffices.
    const int pb = o & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      smM[pb][wv][r][lane] = M[r];
      smS[pb][wv][r][lane] = S[r];
    }
    __syncthreads();
    Lse2<float> tot;
    tot.m = smM[pb][0][wv][lane];
    tot.s = smS[pb][0][wv][lane];
#pragma unroll
    for (int k = 1; k < 4; ++k) tot.merge(smM[pb][k][wv][lane], smS[pb][k][wv][lane]);
    if (valid) epi_apply<float>(eo, tot.result(), xin, c, side, ep, ra);
    eo = eo_next;
    xin = xin_next;
  }
  epi_finish<float>(ep, ra, (int)lid);
  if (hosting) ctl_reduce_finish(ep.host_ctl, hsnap, hm, hden, hnum, hdu, ep.host_hist, par);
}

// output tiles per block: 1 unless there are enough line groups to fill the
// chip with fewer, longer blocks, and only while one chunk of tap tiles
// holds all of a wave's tiles (so the taps are loaded once per block)
static inline int tf_tpc(int n) {
  const int per_wave = (n / 16 + 3) / 4;
  return per_wave >= 4 ? 4 : (per_wave >= 2 ? 2 : 1);
}

static inline int tf_opb(int n, int64_t groups) {
  const int nt = n / 16;
  if (nt > 4 * tf_tpc(n)) return 1;
  int opb = 1;
  while (nt % (opb * 2) == 0 && (int64_t)(nt / (opb * 2)) * groups >= 2048) opb *= 2;
  return opb;
}

static inline int64_t tf_groups(int64_t A, int64_t B, bool strided) {
  return strided ? A * ((B + 15) / 16) : (A + 15) / 16;
}

int grid_tf_parts(int n, int64_t A, int64_t B, bool strided) {
  const int64_t g = tf_groups(A, B, strided);
  return (int)((n / 16) / tf_opb(n, g) * g);
}

template <bool ST, int TP, bool HF>
static void launch_tf_t(unsigned blocks, int opb, const float* in, int64_t A, int n, int64_t B, double h, int side,
                        const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  if (opb > 1)
    hipLaunchKernelGGL((k_grid_tf<ST, TP, true, HF>), dim3(blocks), dim3(kBlock), 0, s, in, n, A, B, opb, h, side, c,
                       ep);
  else
    hipLaunchKernelGGL((k_grid_tf<ST, TP, false, HF>), dim3(blocks), dim3(kBlock), 0, s, in, n, A, B, 1, h, side, c,
                       ep);
}

template <bool ST, bool HF>
static void launch_tf_tpc(int tpc, unsigned blocks, int opb, const float* in, int64_t A, int n, int64_t B, double h,
                          int side, const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  if (tpc == 4) launch_tf_t<ST, 4, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
  else if (tpc == 2) launch_tf_t<ST, 2, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
  else launch_tf_t<ST, 1, HF>(blocks, opb, in, A, n, B, h, side, c, ep, s);
}

void launch_grid_tf(const float* in, int64_t A, int n, int64_t B, bool strided, bool half, double h, int side,
                    const Ctrl* c, const EpiArgs<float>& ep, hipStream_t s) {
  const int64_t g = tf_groups(A, B, strided);
  const int opb = tf_opb(n, g);
  const unsigned blocks = (unsigned)((n / 16) / opb * g);
  const int tpc = tf_tpc(n);
  if (strided) {
    if (half) launch_tf_tpc<true, true>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
    else launch_tf_tpc<true, false>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
  } else {
    if (half) launch_tf_tpc<false, true>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
    else launch_tf_tpc<false, false>(tpc, blocks, opb, in, A, n, B, h, side, c, ep, s);
  }
}

}  // namespace uot
