// Backward of the render (recompute-based): per tile, the forward
// front-to-back pass is replayed with identical FP32 decisions and the
// gradient of every contributing (splat, pixel) pair is formed on the fly,
// using the final pixel colour to obtain the colour behind each splat.  Each
// (splat, tile) instance gets one partial of per-pixel sums (moments about the
// tile centre, dL/do, dL/dRGB), written at its emission index without
// atomics.  The projection backward then forms each drawn splat's 2D sums
// from its partials in FP64 and carries them through the conic inverse, the
// EWA Jacobian, the camera transform, the covariance factorisation, the
// quaternion normalisation, the sigmoid and the SH basis to the raw
// parameters.
#include "lodgs_internal.h"
#include "lodgs_proj.h"

namespace lodgs {

// Reduce-scatter of NP (10 or 11) per-lane values inside each 16-lane row (all lanes
// active): four DPP exchange steps pair lane l with l^1, l^2, l^7 and l^15;
// at each step a lane keeps half of its remaining values (chosen by b0^b2,
// b1^b2, b2^b3 and b3 of l & 15) and adds its partner's copy of that half.
// Lane l then holds its row's sum of value
// slot(l) = (b0^b2) + 2 (b1^b2) + 4 (b2^b3) + 8 b3 (slots NP..15 are zero).
#define LODGS_DPP(x, ctrl) __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xf, 0xf, false))
#define LODGS_RS_PAIR(out, a, b, k, ctrl)       \
  do {                                          \
    const float keep_ = (k) ? (b) : (a);        \
    const float send_ = (k) ? (a) : (b);        \
    (out) = keep_ + LODGS_DPP(send_, ctrl);     \
  } while (0)

template <int NP>
__device__ __forceinline__ float row_reduce_scatter(const float* g, int lane, int& slot) {
  static_assert(NP == 10 || NP == 11, "10 or 11 values");
  const int b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  const bool k1 = (b0 ^ b2) != 0, k2 = (b1 ^ b2) != 0, k3 = (b2 ^ b3) != 0, k4 = b3 != 0;
  float h0, h1, h2, h3, h4, h5;
  LODGS_RS_PAIR(h0, g[0], g[1], k1, 0xB1);  // quad_perm [1,0,3,2]: l^1
  LODGS_RS_PAIR(h1, g[2], g[3], k1, 0xB1);
  LODGS_RS_PAIR(h2, g[4], g[5], k1, 0xB1);
  LODGS_RS_PAIR(h3, g[6], g[7], k1, 0xB1);
  LODGS_RS_PAIR(h4, g[8], g[9], k1, 0xB1);
  if (NP == 11) LODGS_RS_PAIR(h5, g[10], 0.0f, k1, 0xB1);
  else h5 = 0.0f;
  float q0, q1, q2;
  LODGS_RS_PAIR(q0, h0, h1, k2, 0x4E);  // quad_perm [2,3,0,1]: l^2
  LODGS_RS_PAIR(q1, h2, h3, k2, 0x4E);
  LODGS_RS_PAIR(q2, h4, h5, k2, 0x4E);
  float r0, r1;
  LODGS_RS_PAIR(r0, q0, q1, k3, 0x141);  // row_half_mirror: l^7
  LODGS_RS_PAIR(r1, q2, 0.0f, k3, 0x141);
  float z;
  LODGS_RS_PAIR(z, r0, r1, k4, 0x140);  // row_mirror: l^15
  slot = (int)k1 + 2 * (int)k2 + 4 * (int)k3 + 8 * (int)k4;
  return z;
}
#undef LODGS_RS_PAIR
#undef LODGS_DPP

// Backward of the blend: the forward's decisions, pixel layout blend_pixel<PX, true>
// (each wave's rows spread over the block rows and columns).
// Each 16-lane row replays only the splats whose forward event bits cover one
// of its blocks: elsewhere no pixel of the row blended the splat or stopped on
// it in the forward, so the replay would leave every value unchanged.  The
// rows of a wave step through their lists together, each on its own splat.
//
// Per pixel, dL/dalpha = T (G . c) - (G . (C - Q)) / (1 - alpha), with G =
// dL/dC, c the splat colour, C the final colour and Q the colour blended up
// to and including the splat; G . C is fixed per pixel and G . Q is kept as
// one running scalar.  With w = dL/dpower = alpha dL/dalpha, the geometric
// part of a splat's gradient needs sum w d and sum w d d^T over its pixels,
// d = pixel - mean.  They are gathered as moments about the tile centre c_t
// (e = pixel - c_t, |e| <= 7.5): sum w, sum w e, sum w e e^T, so the FP32
// sums stay well conditioned even for a splat whose mean lies far off the
// screen; the projection backward shifts them by c_t - mean in FP64.  Per
// step, each row reduces these NP values of its splat (moments, dL/do, the
// colour gradient and, with NP = 11, the number of pixels it contributes to)
// over its lanes (only when some lane of the wave
// contributes) and adds them to its wave's LDS row of that splat, the four
// rows with one LDS add instruction (the LDS applies the lanes of one
// instruction in lane order, so two rows on the same splat add in row order,
// as adding them one after another does); the workgroup then sums the waves'
// rows in order and writes one NP-float partial per (splat, tile) instance at
// the instance's emission index, with zeros for instances that no pixel
// reached.  No order depends on timing: the result is deterministic.
template <int PX, int NP>
__global__ void __launch_bounds__(256 / PX) k_blend_bwd(const ViewConst* __restrict__ vp,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ ival,
                                                        const uint2* __restrict__ info_k,
                                                        const Splat* __restrict__ splats, const FrameCounters* ctr,
                                                        const float* __restrict__ rgb, const float* __restrict__ dL,
                                                        const uint32_t* __restrict__ event,
                                                        const uint32_t* __restrict__ tile_order,
                                                        float* __restrict__ partial) {
  // NB instances per batch: at most one per thread, and at most 128, which
  // keeps the per-wave LDS rows small enough for several workgroups per CU
  constexpr int NT = 256 / PX, NW = 4 / PX, NB = NT < 128 ? NT : 128;
  const ViewConst v = *vp;
  // the first 12 floats of each splat record (mean, axis, power, opacity,
  // colour): all a replay reads, at a 12-word stride that spreads the rows'
  // reads of different slots over the banks
  struct BatchRec {
    float4 a, b, c;
  };
  __shared__ BatchRec batch[NB];
  __shared__ uint32_t bid[NB];
  __shared__ uint32_t ev[NB];
  __shared__ uint8_t hits[NW][4][NB];  // per row of each wave: the batch slots it replays, in order
  // a row of acc per partial component; slot j's component c sits at column
  // j ^ c, so the ten lanes of a row adding one slot's components hit ten
  // banks (the rows are 128 words apart)
  __shared__ float acc[NW][NP][NB];
  __shared__ uint32_t wave_active[NW];  // per wave: some pixel still blends
  const int tile = (int)tile_order[blockIdx.x];
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, row = lane >> 4;
  int px = 0;
  float fy[PX], T[PX], GQ[PX], GC[PX], G0[PX], G1[PX], G2[PX];
  float ey[PX], exx[PX], exy[PX], eyy[PX];  // offsets from the tile centre
  bool live[PX];
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    int py;
    blend_pixel<PX, true>(tx, ty, wv, lane, p, px, py);
    fy[p] = (float)py + 0.5f;
    live[p] = px < v.width && py < v.height;
    T[p] = 1.0f;
    GQ[p] = GC[p] = G0[p] = G1[p] = G2[p] = 0.0f;
    if (live[p]) {
      const int64_t o = 3 * ((int64_t)py * v.width + px);
      G0[p] = dL[o];
      G1[p] = dL[o + 1];
      G2[p] = dL[o + 2];
      GC[p] = __builtin_fmaf(G2[p], rgb[o + 2], __builtin_fmaf(G1[p], rgb[o + 1], G0[p] * rgb[o]));
    }
  }
  const float fx = (float)px + 0.5f;
  const float ex = fx - (float)(16 * tx + 8);
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    ey[p] = fy[p] - (float)(16 * ty + 8);
    exx[p] = ex * ex;
    exy[p] = ex * ey[p];
    eyy[p] = ey[p] * ey[p];
  }
  const uint2 rg = ranges[tile];
  const uint32_t nr = (uint32_t)ctr->n_render;
  const float thr = 1.0f / 255.0f;
  for (int t = threadIdx.x; t < NW * NP * NB; t += NT) (&acc[0][0][0])[t] = 0.0f;
  // The last NB threads load: thread NT - NB + j holds batch slot j, the
  // words (emission index, splat, event word) of this batch and the next, and
  // the splat record of this batch (only for an instance with events: the
  // others are never replayed), so the loads overlap the replay of the batch
  // before.  The first threads write the partials out after a replay, so with
  // four waves the staging of the next batch and the write-out of the last
  // run on different waves.
  const int ld = (int)threadIdx.x - (NT - NB);  // the loaded slot (loaders only)
  const bool loader = ld >= 0;
  auto words = [&](uint32_t b, uint32_t& e, uint32_t& i, uint32_t& w) {
    const uint32_t k = b + (uint32_t)ld;
    e = i = w = 0u;
    if (loader && k < rg.y) {
      e = ival[k];
      i = info_k[k].x;
      w = event[k];
    }
  };
  auto record = [&](uint32_t i, uint32_t w, float4& a, float4& b, float4& c) {
    a = b = c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (w != 0u && i < nr) {  // i >= nr only follows an instance overflow (no events)
      const float4* r = reinterpret_cast<const float4*>(splats + i);
      a = r[0];
      b = r[1];
      c = r[2];
    }
  };
  uint32_t e0, i0, w0, e1, i1, w1;
  words(rg.x, e0, i0, w0);
  words(rg.x + NB, e1, i1, w1);
  float4 ra, rb, rc;
  record(i0, w0, ra, rb, rc);
  uint32_t b0 = rg.x;
  for (; b0 < rg.y; b0 += NB) {
    bool active = false;
#pragma unroll
    for (int p = 0; p < PX; ++p) active = active || live[p];
    // each wave publishes whether a pixel of it still blends with the batch,
    // behind the batch's barrier (no block-wide count, which takes three)
    const bool wave_act = __any(active);
    if (lane == 0) wave_active[wv] = wave_act ? 1u : 0u;
    if (loader) {
      bid[ld] = e0;
      ev[ld] = event_blocks(w0);
      float4* dst = reinterpret_cast<float4*>(&batch[ld]);  // mean, axis, power, opacity, colour
      dst[0] = ra;
      dst[1] = rb;
      dst[2] = rc;
    }
    __syncthreads();
    uint32_t block_act = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) block_act |= wave_active[w];
    if (block_act == 0u) break;  // every pixel of the tile has stopped (the same flags for all threads)
    // the words of the slot this thread writes out after the replay, read
    // now: a loader may stage the next batch while the write-out runs
    const uint32_t out_bid = bid[threadIdx.x % NB], out_ev = ev[threadIdx.x % NB];
    record(i1, w1, ra, rb, rc);
    uint32_t e2, i2, w2;
    words(b0 + 2 * NB, e2, i2, w2);
    const int m = (int)min((uint32_t)NB, rg.y - b0);
    // every row's list of the batch slots whose events meet its blocks, in
    // slot order (ballot ranks); each lane reads its slots' event words once
    // for the four rows
    static_assert(NB % 64 == 0, "whole waves of batch slots");
    uint32_t evw[NB / 64];
#pragma unroll
    for (int c = 0; c < NB / 64; ++c) {
      const int j = c * 64 + lane;
      evw[c] = j < m ? ev[j] : 0u;
    }
    const uint64_t lt = lanemask_lt();
    int nh[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t want = blend_row_blocks<PX, true>(wv, r);
      int cnt = 0;
#pragma unroll
      for (int c = 0; c < NB / 64; ++c) {
        const bool h = (evw[c] & want) != 0u;
        const uint64_t hb = __ballot(h);
        if (h) hits[wv][r][cnt + __popcll(hb & lt)] = (uint8_t)(c * 64 + lane);
        cnt += __popcll(hb);
      }
      nh[r] = cnt;
    }
    // the hit lists are the wave's own (its LDS operations run in order): a
    // wave-level fence and barrier order their writes before the reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int n = row == 0 ? nh[0] : (row == 1 ? nh[1] : (row == 2 ? nh[2] : nh[3]));  // this row's list
    const int nmax = max(max(nh[0], nh[1]), max(nh[2], nh[3]));
    if (__any(active) && nmax > 0) {  // wave-uniform
      // one splat (batch slot j of this row's list; has = false past its end)
      // against the row's pixels; true when every pixel of the wave has
      // stopped
      auto step = [&](const Splat& s, int j, bool has) -> bool {
        float dxs[PX], dys[PX], u1s[PX], u2s[PX], es[PX], oes[PX], als[PX], tts[PX];
        bool cons[PX];
        bool any_con = false, act = false;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
          const float power = splat_power(s, fx, fy[p], dxs[p], dys[p], u1s[p], u2s[p]);
          es[p] = fexp(power);
          oes[p] = s.o * es[p];
          als[p] = fminf(0.99f, oes[p]);
          tts[p] = T[p] * (1.0f - als[p]);
          const bool hit = live[p] & has & (als[p] >= thr);
          const bool stop = hit & (tts[p] < 0.0001f);
          cons[p] = hit & !stop;
          live[p] = live[p] & !stop;
          any_con = any_con | cons[p];
          act = act | live[p];
        }
        if (__any(any_con)) {  // wave-uniform
          // the first pixel's terms start the sums: only the sign of a zero
          // sum differs from adding them to +0, and the LDS rows (never -0)
          // absorb that
          float g[11];
#pragma unroll
          for (int p = 0; p < PX; ++p) {
            const float alpha = als[p], Tp = T[p];
            const float w = alpha * Tp;
            const float Gc = __builtin_fmaf(G2[p], s.b, __builtin_fmaf(G1[p], s.g, G0[p] * s.r));
            const float gq = __builtin_fmaf(w, Gc, GQ[p]);
            const float ia = __builtin_amdgcn_rcpf(1.0f - alpha);  // gradient values only
            const float dA = Tp * Gc - (GC[p] - gq) * ia;
            const bool con = cons[p];
            const bool unclamped = con & (oes[p] <= 0.99f);
            // the factors are zeroed for pixels without a contribution (the
            // other factors are finite), so the sums need no further selects
            const float dpow = unclamped ? dA * alpha : 0.0f;
            const float dop = unclamped ? dA * es[p] : 0.0f;
            const float wc = con ? w : 0.0f;
            if (p == 0) {
              g[0] = dpow;
              g[1] = dpow * ex;
              g[2] = dpow * ey[p];
              g[3] = dpow * exx[p];
              g[4] = dpow * exy[p];
              g[5] = dpow * eyy[p];
              g[6] = dop;
              g[7] = G0[p] * wc;
              g[8] = G1[p] * wc;
              g[9] = G2[p] * wc;
              g[10] = con ? 1.0f : 0.0f;  // contributing pixels (read only with NP = 11)
            } else {
              g[0] += dpow;
              g[1] = __builtin_fmaf(dpow, ex, g[1]);
              g[2] = __builtin_fmaf(dpow, ey[p], g[2]);
              g[3] = __builtin_fmaf(dpow, exx[p], g[3]);
              g[4] = __builtin_fmaf(dpow, exy[p], g[4]);
              g[5] = __builtin_fmaf(dpow, eyy[p], g[5]);
              g[6] += dop;
              g[7] = __builtin_fmaf(G0[p], wc, g[7]);
              g[8] = __builtin_fmaf(G1[p], wc, g[8]);
              g[9] = __builtin_fmaf(G2[p], wc, g[9]);
              if (NP == 11) g[10] += con ? 1.0f : 0.0f;
            }
            GQ[p] = con ? gq : GQ[p];
            T[p] = con ? tts[p] : Tp;
          }
          int slot;
          const float r = row_reduce_scatter<NP>(g, lane, slot);
          // the rows add into the wave's row of their splats with one LDS
          // add instruction (two rows may be on the same splat: the LDS
          // applies the lanes of one instruction in a fixed order)
          const uint64_t cm = __ballot(any_con);
          if (slot < NP && ((cm >> (16 * row)) & 0xFFFFull) != 0ull)
            __hip_atomic_fetch_add(&acc[wv][slot][j ^ slot], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        return !__any(act);
      };
      // two register sets, each loaded one list entry ahead of its use
      static_assert((NB & (NB - 1)) == 0, "a power of two of list entries");
      const uint8_t* hl = hits[wv][row];
      // (an entry is read unconditionally, within the row's NB bytes, and
      // replaced by 0 past the list's end, so every read is a plain LDS load)
      auto slot_at = [&](int t) -> int {
        const int e = (int)hl[t & (NB - 1)];
        return t < n ? e : 0;
      };
      auto rec = [&](int j) -> Splat {
        const BatchRec& q = batch[j];
        Splat sp;
        sp.mxh = q.a.x;
        sp.mxl = q.a.y;
        sp.myh = q.a.z;
        sp.myl = q.a.w;
        sp.ce = q.b.x;
        sp.se = q.b.y;
        sp.h1 = q.b.z;
        sp.h2 = q.b.w;
        sp.o = q.c.x;
        sp.r = q.c.y;
        sp.g = q.c.z;
        sp.b = q.c.w;
        sp.rect_x = sp.rect_y = sp.pad0 = sp.pad1 = 0u;
        return sp;
      };
      // (the list entries themselves two ahead, so a record's LDS read never
      // waits for the read of its slot index)
      int ja = slot_at(0), jb = slot_at(1);
      Splat sa = rec(ja), sb;
      for (int t = 0;;) {
        const int jc = slot_at(t + 2);
        sb = rec(jb);
        if (step(sa, ja, t < n) || ++t >= nmax) break;
        const int jd = slot_at(t + 2);
        sa = rec(jc);
        if (step(sb, jb, t < n) || ++t >= nmax) break;
        ja = jc;
        jb = jd;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      // Only the waves whose blocks hold one of the instance's events replayed
      // it: the other waves' rows of this slot are still +0 and are neither
      // read nor cleared.  Skipping them leaves the sums bit-identical (a row
      // value is never -0: rows start at +0 and x + y is -0 only when both
      // are), and an instance without events is written as zeros.
      float* dst = partial + NP * (int64_t)out_bid;
      const uint32_t evb = out_ev;
      float r[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) r[c] = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        uint32_t wb = 0u;
#pragma unroll
        for (int g = 0; g < 4; ++g) wb |= blend_row_blocks<PX, true>(w, g);
        if ((evb & wb) == 0u) continue;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          const int col = (int)threadIdx.x ^ c;
          r[c] += acc[w][c][col];
          acc[w][c][col] = 0.0f;
        }
      }
#pragma unroll
      for (int c = 0; c < NP; ++c) dst[c] = r[c];
    }
    e0 = e1;
    i0 = i1;
    w0 = w1;
    e1 = e2;
    i1 = i2;
    w1 = w2;
  }
  // instances that no pixel of the tile reached
  for (uint32_t k = b0 + threadIdx.x; k < rg.y; k += NT) {
    float* dst = partial + NP * (int64_t)ival[k];
#pragma unroll
    for (int c = 0; c < NP; ++c) dst[c] = 0.0f;
  }
}

// Projection backward, FP64 (per splat): the forward chain is replayed and the
// 2D gradients (mean2D, conic, opacity, colour) are carried to the raw
// parameters.
// Zeroes the per-selection gradient rows (splats that were not drawn keep 0):
// each group's rows [0, n_render) are one contiguous span, cleared with
// consecutive lanes on consecutive words.
__global__ void __launch_bounds__(kBlock) k_zero_sel(const FrameCounters* ctr, int nc, lodgs_grads sel) {
  const int64_t n = ctr->n_render;
  float* const arr[5] = {sel.d_means, sel.d_log_scales, sel.d_quats, sel.d_opacity_logits, sel.d_sh};
  const int w[5] = {3, 3, 4, 1, nc};
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  for (int g = 0; g < 5; ++g) {
    float* a = arr[g];
    if (!a) continue;
    for (int64_t e = t0; e < n * w[g]; e += stride) a[e] = 0.0f;
  }
}

// Every real SH basis function of degree <= 3 is C L Q with a linear
// monomial L = lx x + ly y + lz z + l1 (one coefficient set) and a quadratic
// form Q = a xx + b yy + g zz + d xy + e yz + f xz + h; row k holds
// (C, lx, ly, lz, l1, a, b, g, d, e, f, h) for basis function k (the same
// functions as sh_basis), so any basis function is evaluated without
// branches.
__constant__ float kShFactors[16][12] = {
    {kSH0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 1},
    {-kSH1, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 1},
    {kSH1, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 1},
    {-kSH1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1},
    {kSH2_0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0},
    {kSH2_1, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0},
    {kSH2_2, 0, 0, 0, 1, -1, -1, 2, 0, 0, 0, 0},
    {kSH2_3, 0, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0},
    {kSH2_4, 0, 0, 0, 1, 1, -1, 0, 0, 0, 0, 0},
    {kSH3_0, 0, 1, 0, 0, 3, -1, 0, 0, 0, 0, 0},
    {kSH3_1, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0},
    {kSH3_2, 0, 1, 0, 0, -1, -1, 4, 0, 0, 0, 0},
    {kSH3_3, 0, 0, 1, 0, -3, -3, 2, 0, 0, 0, 0},
    {kSH3_4, 1, 0, 0, 0, -1, -1, 4, 0, 0, 0, 0},
    {kSH3_5, 0, 0, 1, 0, 1, -1, 0, 0, 0, 0, 0},
    {kSH3_6, 1, 0, 0, 0, 1, -3, 0, 0, 0, 0, 0},
};

// Real SH basis function k at the unit direction (x, y, z).
__device__ __forceinline__ float sh_basis_value(int k, float x, float y, float z) {
  const float* t = kShFactors[k];
  const float L = __builtin_fmaf(t[1], x, __builtin_fmaf(t[2], y, __builtin_fmaf(t[3], z, t[4])));
  float Q = t[11];
  Q = __builtin_fmaf(t[5] * x, x, Q);
  Q = __builtin_fmaf(t[6] * y, y, Q);
  Q = __builtin_fmaf(t[7] * z, z, Q);
  Q = __builtin_fmaf(t[8] * x, y, Q);
  Q = __builtin_fmaf(t[9] * y, z, Q);
  Q = __builtin_fmaf(t[10] * x, z, Q);
  return t[0] * L * Q;
}

// One instance's partial (moments about its tile's centre, dL/do, colour
// gradient) as the splat's 2D sums in FP64: with D = c_t - mean,
//   sum w d = m1 + D m0,  sum w d d^T = m2 + D m1^T + m1 D^T + D D^T m0,
// added into g = [sum w dx, sum w dy, sum w dx^2, sum w dx dy, sum w dy^2,
// dL/do, dL/dr, dL/dg, dL/db, contributing pixels].  l is the instance's index within its splat,
// whose tiles it enumerates row by row over the rectangle q.
template <int NP>
__device__ __forceinline__ void add_instance(double* g, const float* P, uint32_t l, ushort4 q, double mx,
                                             double my) {
  const uint32_t w = (uint32_t)(q.y - q.x);
  const uint32_t tyy = w ? (uint32_t)q.z + l / w : 0u, txx = w ? (uint32_t)q.x + l % w : 0u;
  const double Dx = (double)(16u * txx + 8u) - mx, Dy = (double)(16u * tyy + 8u) - my;
  const double m0 = P[0], m1x = P[1], m1y = P[2];
  g[0] += m1x + Dx * m0;
  g[1] += m1y + Dy * m0;
  g[2] += (double)P[3] + 2.0 * Dx * m1x + Dx * Dx * m0;
  g[3] += (double)P[4] + Dx * m1y + Dy * m1x + Dx * Dy * m0;
  g[4] += (double)P[5] + 2.0 * Dy * m1y + Dy * Dy * m0;
#pragma unroll
  for (int c = 5; c < NP - 1; ++c) g[c] += (double)P[c + 1];
}

__device__ __forceinline__ void splat_mean64(const Splat* splats, int64_t i, double& mx, double& my) {
  const float4 m = *reinterpret_cast<const float4*>(&splats[i].mxh);  // mxh, mxl, myh, myl
  mx = (double)m.x + (double)m.y;
  my = (double)m.z + (double)m.w;
}

// Splats with more than kLongSegment instances: one workgroup per splat turns
// its instance partials into the splat's 2D sums (add_instance) in grad2d at
// its selection position (and its contributing pixels in contrib).  Per-thread FP64 sums over independent unrolled loads, a
// butterfly over the wave, the waves in order: a fixed order, so
// deterministic.
template <int NP>
__global__ void __launch_bounds__(kBlock) k_long_sums(const FrameCounters* ctr, const uint32_t* long_list,
                                                      const uint32_t* order,
                                                      const uint32_t* inst_off, const float* __restrict__ partial,
                                                      const Splat* __restrict__ splats, const ushort4* rect,
                                                      double* grad2d, int32_t* contrib) {
  __shared__ double part[kBlock / 64][10];
  const int64_t n = ctr->n_drawn, nl = ctr->n_long;
  const int64_t n_inst = (uint32_t)ctr->n_instances, n_cl = ctr->n_inst_clamped;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t li = blockIdx.x; li < nl; li += gridDim.x) {  // block-uniform
    const int64_t r = long_list[li];
    const int64_t i = order[r];
    const int64_t a0 = inst_off[r];
    int64_t a = a0, b = r + 1 < n ? (int64_t)inst_off[r + 1] : n_inst;
    a = a < n_cl ? a : n_cl;
    b = b < n_cl ? b : n_cl;
    const ushort4 q = rect[i];
    double mx, my;
    splat_mean64(splats, i, mx, my);
    double g[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t q0 = a + threadIdx.x; q0 < b; q0 += 4 * kBlock) {
      float t[4][NP];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = q0 + (int64_t)u * kBlock;
#pragma unroll
        for (int c = 0; c < NP; ++c) t[u][c] = k < b ? partial[NP * k + c] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = q0 + (int64_t)u * kBlock;
        if (k < b) add_instance<NP>(g, t[u], (uint32_t)(k - a0), q, mx, my);
      }
    }
#pragma unroll
    for (int c = 0; c < 10; ++c)
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) g[c] += __shfl_xor(g[c], d, 64);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 10; ++c) part[wv][c] = g[c];
    }
    __syncthreads();
    if (threadIdx.x < 10) {
      double sum = part[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) sum += part[w][threadIdx.x];
      if (threadIdx.x < 9) grad2d[9 * i + threadIdx.x] = sum;
      else if (NP == 11) contrib[i] = (int32_t)sum;  // a count, exact in FP64
    }
    __syncthreads();
  }
}

// Every drawn splat that the duplication kernel did not put on the long list
// (those with more than kLongSegment tiles whose first instance was emitted):
// one thread per splat, in depth order, so neighbouring threads read
// neighbouring partials; FP64 sums in instance order (add_instance) into
// grad2d at the splat's selection position (zero for a splat that an
// instance overflow left without instances), and its number of contributing
// pixels into contrib.
template <int NP>
__global__ void __launch_bounds__(kBlock) k_splat_sums(const FrameCounters* ctr, const uint32_t* order,
                                                       const uint32_t* inst_off,
                                                       const float* __restrict__ partial,
                                                       const Splat* __restrict__ splats, const ushort4* rect,
                                                       const uint4* rank_info, double* grad2d, int32_t* contrib) {
  const int64_t n = ctr->n_drawn;
  const int64_t n_inst = (uint32_t)ctr->n_instances, n_cl = ctr->n_inst_clamped;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = inst_off[r];
    int64_t i;
    ushort4 q;
    double mx, my;
    if (a0 < n_cl) {  // the duplication kernel wrote the rank's record with the first instance
      const uint4 w0 = rank_info[2 * r], w1 = rank_info[2 * r + 1];
      i = w0.x;
      q = make_ushort4((unsigned short)(w0.z & 0xFFFFu), (unsigned short)(w0.z >> 16),
                       (unsigned short)(w0.w & 0xFFFFu), (unsigned short)(w0.w >> 16));
      mx = (double)__uint_as_float(w1.x) + (double)__uint_as_float(w1.y);
      my = (double)__uint_as_float(w1.z) + (double)__uint_as_float(w1.w);
    } else {  // left without instances by an overflow: zero sums
      i = order[r];
      q = rect[i];
      mx = my = 0.0;
    }
    if ((uint32_t)(q.y - q.x) * (uint32_t)(q.w - q.z) > kLongSegment && a0 < n_cl) continue;  // k_long_sums
    int64_t b = r + 1 < n ? (int64_t)inst_off[r + 1] : n_inst;
    const int64_t a = a0 < n_cl ? a0 : n_cl;
    b = b < n_cl ? b : n_cl;
    double g[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t k = a; k < b; ++k) {
      float t[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) t[c] = partial[NP * k + c];
      add_instance<NP>(g, t, (uint32_t)(k - a0), q, mx, my);
    }
    double* dst = grad2d + 9 * i;
#pragma unroll
    for (int c = 0; c < 9; ++c) dst[c] = g[c];
    if (NP == 11) contrib[i] = (int32_t)g[9];
  }
}

// Per drawn splat, 16 lanes, in selection order (ascending node index, so
// neighbouring groups read neighbouring nodes): the colour backward.  dL/dRGB
// (the splat's colour sums in grad2d; zero for a channel the forward clamped
// at 0, a decision the forward recorded) goes to the SH coefficients, lane k
// taking basis function k (contiguous reads and writes of the 192-byte
// coefficient block), and, through the forward's d colour / d direction, to
// the view direction; dL/dmean through the view direction then replaces the
// colour sums in grad2d.  The forward's per-splat record holds the view
// direction, 1 / distance and the clamp bits, so no node parameter but the
// coefficients is read.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_color_bwd(const int32_t* idx, const FrameCounters* ctr,
                                                      const uint32_t* drawn_list, const float* __restrict__ dcol,
                                                      double* grad2d, float* sel_sh, float* node_sh) {
  constexpr int nb = (DEG + 1) * (DEG + 1), nc = 3 * nb;
  const int64_t n = ctr->n_drawn;
  const int lane = threadIdx.x & 63, sub = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t g0 = wave * 4; g0 < n; g0 += waves * 4) {  // wave-uniform
    const int64_t dr = g0 + (lane >> 4);  // drawn rank
    if (dr >= n) continue;
    const int64_t i = drawn_list[dr];
    float gc[3], acc3[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 3; ++c) gc[c] = (float)grad2d[9 * i + 6 + c];
    const float4* rec = reinterpret_cast<const float4*>(dcol + kColorRec * i);
    const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3];
    const float J[9] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x};
    const float d0 = r2.y, d1 = r2.z, d2 = r2.w, il = r3.x;
    const uint32_t clamp = __float_as_uint(r3.y);
    const int64_t node = idx[i];
    // rows of 12 or 48 floats (degree 1 or 3) move as float4s: lane q takes
    // floats 4q .. 4q + 3 of the row, coefficient f / 3 and channel f % 3 of
    // float f; other degrees move one coefficient (3 floats) per lane
    constexpr bool kVec = nc % 4 == 0;
    constexpr int nq = nc / 4;
    float4 acc4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (kVec) {
      if (node_sh && sub < nq) acc4 = *reinterpret_cast<const float4*>(node_sh + (int64_t)nc * node + 4 * sub);
    } else if (node_sh && sub < nb) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc3[c] = node_sh[(int64_t)nc * node + 3 * sub + c];
    }
    // gradient values only: FP32 throughout
    const float dRGB[3] = {(clamp & 1u) ? 0.0f : gc[0], (clamp & 2u) ? 0.0f : gc[1], (clamp & 4u) ? 0.0f : gc[2]};
    const float Yk = sub < nb ? sh_basis_value(sub, d0, d1, d2) : 0.0f;
    if (kVec) {
      float gk[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {  // every lane of the row takes part in the shuffles
        const int f = 4 * sub + t;
        const int k = f / 3 < nb ? f / 3 : nb - 1, c = f - 3 * (f / 3);
        const float Yf = __shfl(Yk, (lane & ~15) + k, 64);
        gk[t] = (c == 0 ? dRGB[0] : (c == 1 ? dRGB[1] : dRGB[2])) * Yf;
      }
      if (sub < nq) {
        if (sel_sh)
          *reinterpret_cast<float4*>(sel_sh + (int64_t)nc * i + 4 * sub) = make_float4(gk[0], gk[1], gk[2], gk[3]);
        if (node_sh)
          *reinterpret_cast<float4*>(node_sh + (int64_t)nc * node + 4 * sub) =
              make_float4(acc4.x + gk[0], acc4.y + gk[1], acc4.z + gk[2], acc4.w + gk[3]);
      }
    } else if (sub < nb) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float gk = dRGB[c] * Yk;
        if (sel_sh) sel_sh[(int64_t)nc * i + 3 * sub + c] = gk;
        if (node_sh) node_sh[(int64_t)nc * node + 3 * sub + c] = acc3[c] + gk;
      }
    }
    if (sub == 0) {  // dL/ddir, projected onto the sphere's tangent plane, / |mu - pos|
      float dd[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        dd[a] = __builtin_fmaf(dRGB[2], J[6 + a], __builtin_fmaf(dRGB[1], J[3 + a], dRGB[0] * J[a]));
      const float dot = __builtin_fmaf(dd[0], d0, __builtin_fmaf(dd[1], d1, dd[2] * d2));
      grad2d[9 * i + 6] = (double)((dd[0] - d0 * dot) * il);
      grad2d[9 * i + 7] = (double)((dd[1] - d1 * dot) * il);
      grad2d[9 * i + 8] = (double)((dd[2] - d2 * dot) * il);
    }
  }
}

// One thread per drawn splat, in selection order (ascending node index, so
// neighbouring lanes touch neighbouring nodes): drawn_list[0 .. n_drawn)
// lists exactly the drawn splats.  The FP64 geometry chain is replayed and
// the 2D gradients of grad2d[r] are carried to the mean, scales, rotation and
// opacity logit; grad2d[r][6..8] already holds dL/dmean through the view
// direction.
template <int DEG>
__global__ void __launch_bounds__(kBlock) k_project_bwd(SceneDev S, const ViewConst* __restrict__ vp, const int32_t* idx,
                                                        const FrameCounters* ctr, const uint32_t* drawn_list,
                                                        const double* grad2d, lodgs_grads sel, lodgs_grads nodes,
                                                        float* max_grad2d, ContribStats cs) {
  const int32_t iter = cs.last ? *cs.iteration : 0;
  const ViewConst v = *vp;
  const int64_t n = ctr->n_drawn;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = drawn_list[r];
    const int64_t node = idx[i];
    if (cs.last) {  // pruning statistics: a drawn node is one splat of its view (no races)
      const int32_t c = cs.contrib[i];
      if (c > 0) {
        cs.last[node] = iter;
        if (cs.count) cs.count[node] += c;
      }
    }
    double g2[9];  // 2D sums of the splat (selection position i), see add_instance
#pragma unroll
    for (int c = 0; c < 9; ++c) g2[c] = grad2d[9 * i + c];
    const double gdir[3] = {g2[6], g2[7], g2[8]};
    double gm[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
    Proj64 P;
    const bool visible = proj_chain64(S.means, S.log_scales, S.quats, v, node, P);
    if (visible) {
      // opacity
      const double o = 1.0 / (1.0 + (double)fexp(-S.opacity_logits[node]));
      go = g2[5] * o * (1.0 - o);
      // d power / d mean2D = Q d, d power / d conic = -(dx^2 / 2, dx dy, dy^2 / 2)
      const double ca = P.C / P.det, cb = -P.B / P.det, cc = P.A / P.det;
      const double gmx = ca * g2[0] + cb * g2[1], gmy = cb * g2[0] + cc * g2[1];
      // the densification statistic: the largest screen-space mean gradient
      // over views (a drawn node is one splat of its view: no races)
      if (max_grad2d) max_grad2d[node] = fmaxf(max_grad2d[node], (float)__builtin_sqrt(gmx * gmx + gmy * gmy));
      // conic -> projected covariance: GS = -Q GQ Q
      const double gq00 = -0.5 * g2[2], gq01 = -0.5 * g2[3], gq11 = -0.5 * g2[4];
      const double qg00 = ca * gq00 + cb * gq01, qg01 = ca * gq01 + cb * gq11;
      const double qg10 = cb * gq00 + cc * gq01, qg11 = cb * gq01 + cc * gq11;
      const double GS00 = -(qg00 * ca + qg01 * cb), GS01 = -(qg00 * cb + qg01 * cc);
      const double GS11 = -(qg10 * cb + qg11 * cc);
      // Sigma' = T Sigma T^T: dL/dT = 2 GS T Sigma, dL/dSigma = T^T GS T
      const double* Tm = P.T;
      const double* Sg = P.Sg;
      double TS[6];
      for (int r = 0; r < 2; ++r) {
        TS[3 * r + 0] = Tm[3 * r] * Sg[0] + Tm[3 * r + 1] * Sg[1] + Tm[3 * r + 2] * Sg[2];
        TS[3 * r + 1] = Tm[3 * r] * Sg[1] + Tm[3 * r + 1] * Sg[3] + Tm[3 * r + 2] * Sg[4];
        TS[3 * r + 2] = Tm[3 * r] * Sg[2] + Tm[3 * r + 1] * Sg[4] + Tm[3 * r + 2] * Sg[5];
      }
      double dT[6];
      for (int c = 0; c < 3; ++c) {
        dT[c] = 2.0 * (GS00 * TS[c] + GS01 * TS[3 + c]);
        dT[3 + c] = 2.0 * (GS01 * TS[c] + GS11 * TS[3 + c]);
      }
      double dS[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          dS[3 * a + b] = Tm[a] * (GS00 * Tm[b] + GS01 * Tm[3 + b]) + Tm[3 + a] * (GS01 * Tm[b] + GS11 * Tm[3 + b]);
      // T = J W
      double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
      for (int c = 0; c < 3; ++c) {
        dJ00 += dT[c] * (double)v.R[c];
        dJ02 += dT[c] * (double)v.R[6 + c];
        dJ11 += dT[3 + c] * (double)v.R[3 + c];
        dJ12 += dT[3 + c] * (double)v.R[6 + c];
      }
      const double cx = P.c[0], cy = P.c[1], cz = P.c[2];
      const double fx = v.fx, fy = v.fy;
      const double iz = 1.0 / cz, iz2 = iz * iz, iz3 = iz2 * iz;
      const double dcx = dJ02 * (-fx * iz2) + gmx * fx * iz;
      const double dcy = dJ12 * (-fy * iz2) + gmy * fy * iz;
      const double dcz = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * cx * iz3) + dJ11 * (-fy * iz2) +
                         dJ12 * (2.0 * fy * cy * iz3) + gmx * (-fx * cx * iz2) + gmy * (-fy * cy * iz2);
      for (int a = 0; a < 3; ++a)
        gm[a] = (double)v.R[a] * dcx + (double)v.R[3 + a] * dcy + (double)v.R[6 + a] * dcz + gdir[a];
      // Sigma = M M^T, M = Rq diag(s)
      double dRq[9];
      for (int c = 0; c < 3; ++c) {
        double ds = 0.0;
        for (int r = 0; r < 3; ++r) {
          const double dm = 2.0 * (dS[3 * r] * P.M[c] + dS[3 * r + 1] * P.M[3 + c] + dS[3 * r + 2] * P.M[6 + c]);
          ds += dm * P.Rq[3 * r + c];
          dRq[3 * r + c] = dm * P.s[c];
        }
        gls[c] = ds * P.s[c];
      }
      const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
      double dq[4];
      dq[0] = 2.0 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
      dq[1] = 2.0 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2.0 * x * dRq[4] - w * dRq[5] + z * dRq[6] +
                     w * dRq[7] - 2.0 * x * dRq[8]);
      dq[2] = 2.0 * (-2.0 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] +
                     z * dRq[7] - 2.0 * y * dRq[8]);
      dq[3] = 2.0 * (-2.0 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2.0 * z * dRq[4] + y * dRq[5] +
                     x * dRq[6] + y * dRq[7]);
      const double qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
      for (int k = 0; k < 4; ++k) gq[k] = (dq[k] - P.qn[k] * qd) / P.ql;
    }
    if (sel.d_means) for (int k = 0; k < 3; ++k) sel.d_means[3 * i + k] = (float)gm[k];
    if (sel.d_log_scales) for (int k = 0; k < 3; ++k) sel.d_log_scales[3 * i + k] = (float)gls[k];
    if (sel.d_quats) for (int k = 0; k < 4; ++k) sel.d_quats[4 * i + k] = (float)gq[k];
    if (sel.d_opacity_logits) sel.d_opacity_logits[i] = (float)go;
    if (!visible) continue;
    if (nodes.d_means) for (int k = 0; k < 3; ++k) nodes.d_means[3 * node + k] += (float)gm[k];
    if (nodes.d_log_scales) for (int k = 0; k < 3; ++k) nodes.d_log_scales[3 * node + k] += (float)gls[k];
    if (nodes.d_quats) for (int k = 0; k < 4; ++k) nodes.d_quats[4 * node + k] += (float)gq[k];
    if (nodes.d_opacity_logits) nodes.d_opacity_logits[node] += (float)go;
  }
}

// The per-splat 2D sums of the instance partials (frame-local outputs).
template <int NP>
static void launch_splat_sums(lodgs_frame* f, hipStream_t st) {
  hipLaunchKernelGGL(k_long_sums<NP>, dim3(1024), dim3(kBlock), 0, st, f->ctr, f->long_list, f->sorted_order,
                     f->inst_off, f->inst_grad, f->splats, f->rect, f->grad2d, f->contrib);
  hipLaunchKernelGGL(k_splat_sums<NP>, dim3(2048), dim3(kBlock), 0, st, f->ctr, f->sorted_order, f->inst_off,
                     f->inst_grad, f->splats, f->rect, f->rank_info, f->grad2d, f->contrib);
}

// Colour and projection backward into the gradient arrays (and the node
// statistics).
template <int DEG>
static void launch_scatter_deg(const SceneDev& S, lodgs_frame* f, const lodgs_grads& sel, const lodgs_grads& nodes,
                               bool contrib, hipStream_t st) {
  // 16 lanes per splat: one pass covers 256k drawn splats, so each 16-lane
  // group runs its latency-bound chain of dependent loads once
  hipLaunchKernelGGL(k_color_bwd<DEG>, dim3(16384), dim3(kBlock), 0, st, f->r_idx, f->ctr, f->drawn_list, f->dcol,
                     f->grad2d, sel.d_sh, nodes.d_sh);
  ContribStats cs{f->contrib, nullptr, nullptr, nullptr};
  if (contrib) cs = ContribStats{f->contrib, f->last_contrib, f->contrib_count, f->contrib_iteration};
  hipLaunchKernelGGL(k_project_bwd<DEG>, dim3(1024), dim3(kBlock), 0, st, S, f->d_view_ren, f->r_idx, f->ctr,
                     f->drawn_list, f->grad2d, sel, nodes, f->rows_mode ? (float*)nullptr : f->max_grad2d, cs);
}

template <int NP>
static void launch_blend_bwd_np(lodgs_frame* f, const float* d_dL, hipStream_t st) {
  const ViewConst& v = f->view;
  const int ntiles = v.tiles_x * v.tiles_y;
  switch (f->blend_px_bwd) {
    case 1:
      hipLaunchKernelGGL((k_blend_bwd<1, NP>), dim3(ntiles), dim3(256), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_ival, f->sorted_info, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_event,
                         f->tile_order, f->inst_grad);
      break;
    case 4:
      hipLaunchKernelGGL((k_blend_bwd<4, NP>), dim3(ntiles), dim3(64), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_ival, f->sorted_info, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_event,
                         f->tile_order, f->inst_grad);
      break;
    default:
      hipLaunchKernelGGL((k_blend_bwd<2, NP>), dim3(ntiles), dim3(128), 0, st, f->d_view_ren, f->ranges,
                         f->sorted_ival, f->sorted_info, f->splats, f->ctr, f->r_rgb, d_dL, f->inst_event,
                         f->tile_order, f->inst_grad);
      break;
  }
}

// LODGS_BWD_PARTIALS: the blend backward and the per-splat 2D sums, which
// write only the frame's own state.  The per-instance partials carry the
// contributing-pixel count (11 values) only while the pruning statistic is
// attached (and not in the rows form).  LODGS_BWD_SCATTER: colour and
// projection backward into the gradient arrays and the node statistics; it
// stamps the pruning statistic only after partials that carried the count.
void launch_backward(lodgs_frame* f, const float* d_dL, const lodgs_grads* sel, const lodgs_grads* nodes,
                     uint32_t phases, hipStream_t st) {
  const bool part = (phases & LODGS_BWD_PARTIALS) != 0, scat = (phases & LODGS_BWD_SCATTER) != 0;
  if (part) {
    f->partials_np = (f->last_contrib && !f->rows_mode) ? kPartial : kPartial - 1;
    stage_begin(f, LODGS_STAGE_BLEND_BWD, st);
    if (f->partials_np == kPartial) launch_blend_bwd_np<kPartial>(f, d_dL, st);
    else launch_blend_bwd_np<kPartial - 1>(f, d_dL, st);
    stage_end(f, st);
  }
  if (!part && !scat) return;
  stage_begin(f, LODGS_STAGE_PROJECT_BWD, st);
  if (part) {
    if (f->partials_np == kPartial) launch_splat_sums<kPartial>(f, st);
    else launch_splat_sums<kPartial - 1>(f, st);
  }
  if (scat) {
    const SceneDev& S = render_params(f);
    const bool contrib = f->partials_np == kPartial && f->last_contrib;
    lodgs_grads none{nullptr, nullptr, nullptr, nullptr, nullptr};
    if (sel) hipLaunchKernelGGL(k_zero_sel, dim3(1024), dim3(kBlock), 0, st, f->ctr, S.n_coef, *sel);
    const lodgs_grads gs = sel ? *sel : none, gn = nodes ? *nodes : none;
    switch (S.sh_degree) {
      case 0: launch_scatter_deg<0>(S, f, gs, gn, contrib, st); break;
      case 1: launch_scatter_deg<1>(S, f, gs, gn, contrib, st); break;
      case 2: launch_scatter_deg<2>(S, f, gs, gn, contrib, st); break;
      default: launch_scatter_deg<3>(S, f, gs, gn, contrib, st); break;
    }
  }
  stage_end(f, st);
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// L1 loss: grad = sign(img - target) / n, loss = sum |img - target| / n.
__global__ void __launch_bounds__(kBlock) k_l1(const float* img, const float* tgt, int64_t n, float* grad,
                                               float* loss) {
  const float inv = 1.0f / (float)n;
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = img[i] - tgt[i];
    grad[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    acc += fabsf(d);
  }
  if (!loss) return;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, acc * inv);
}

__global__ void k_zero_one(float* p) { *p = 0.0f; }

int l1_target_arg(const void* func, int* n_args) {
  if (func != reinterpret_cast<const void*>(&k_l1)) return -1;
  *n_args = 5;  // (img, tgt, n, grad, loss)
  return 1;
}

void launch_l1_loss(const float* img, const float* target, int64_t n, float* grad, float* loss, hipStream_t st) {
  if (loss) hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(1), 0, st, loss);
  int64_t g = (n + kBlock - 1) / kBlock;
  g = g > 4096 ? 4096 : g;
  hipLaunchKernelGGL(k_l1, dim3((int)g), dim3(kBlock), 0, st, img, target, n, grad, loss);
}

}  // namespace lodgs
