// The arguments of the single-matrix product kernels and the two-slice
// single-vector product (sec. 4.4) that both the single-matrix and the
// batched products run.
#pragma once

#include "rowdot.hpp"

namespace pksell {

constexpr int kPairBlock = 128;  // threads per workgroup of the two-slice kernels

struct SpmvArgs {
  const uint32_t *pack;
  const int64_t *offset;
  const void *perm;
  const int16_t *row_exp;
  const float *x;
  float *y;
  uint32_t n, m, n_slices;
  int32_t C, perm_bytes, k, r0;
  RowGeo geo;
  Codec cd;
  int32_t group;  // two-slice kernels: words per group (host side only)
  bool resident;  // k = 1, streamed words: cache_hint PKSELL_CACHE_RESIDENT (host side only)
};

// The two-slice single-vector product (C = 64, k = 1) of one wave: slices
// k0 and k0 + 1 of the matrix in ``a`` (k0 < n_slices; a second slice past
// the end reads no words and stores nothing), lane ``lane``.  G words per
// group and slice: the host sizes it to the matrix's slice width (every
// word of a group issues a load and a gather, padding or not, each a full
// 64-lane instruction).  RES: words loaded with the default policy
// (cache_hint RESIDENT).
template <int FMT, bool BUF, bool IMPL, int G, bool RES>
__device__ inline void pair_product(const SpmvArgs &a, uint32_t k0, uint32_t lane) {
  constexpr int S = 2;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.x, a.m * 4u);
  // destinations (implicit order) and FIX row exponents, read up front
  // through range-checked loads
  constexpr bool kFix = FMT == PKSELL_FIX;
  RowOut ro[S];
  if constexpr (IMPL || kFix) {
#pragma unroll
    for (int i = 0; i < S; ++i)
      ro[i] = row_out<FMT>(IMPL ? a.perm : nullptr, a.perm_bytes, a.row_exp,
                           (k0 + i) * kWave + lane, a.n, a.geo);
  }
  int64_t off[S + 1];
#pragma unroll
  for (int i = 0; i <= S; ++i) off[i] = a.offset[min(k0 + i, a.n_slices)];
  uint32_t w[S], c[S], wm = 0;
  float acc[S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    w[i] = (uint32_t)((off[i + 1] - off[i]) >> 6);
    wm = max(wm, w[i]);
    c[i] = left_offset32((k0 + i) * kWave + lane, a.geo);
    acc[i] = 0.0f;
  }
  __amdgpu_buffer_rsrc_t rs[S];
#pragma unroll
  for (int i = 0; i < S; ++i) rs[i] = slice_words(a.pack + off[i], w[i]);
  // Groups of G words per slice.  Streamed loads need no branch (words past
  // a slice's width read 0 from its resource, with no request), which lets
  // each gather go out as soon as its word has arrived instead of after the
  // whole group.  With more than one group, the next group's words are
  // requested before this group's gathers, so the word stream stays in
  // flight while the wave waits on x.
  auto load = [&](uint32_t j, uint32_t (&p)[S][G]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int q = 0; q < G; ++q) {
        uint32_t wd = 0u;  // past the slice's width: a padding word
        if (BUF)
          wd = stream_word<word_policy<RES>()>(rs[i], lane, j + q);
        else if (j + q < w[i])
          wd = __builtin_nontemporal_load(a.pack + off[i] + lane + (j + q) * kWave);
        p[i][q] = wd;
      }
  };
  auto gather = [&](const uint32_t (&p)[S][G], float (&v)[S][G], float (&xv)[S][G]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const Unpacked u = unpack(p[i][q], a.cd);
        c[i] += u.delta;
        v[i][q] = decode_value<FMT>(u.vbits);
        xv[i][q] = buffer_load_f32(rx, (p[i][q] & 1u) ? c[i] << 2 : a.m * 4u);
      }
  };
  // (Groups of 7 or 8 words keep the plain order: the extra G words of
  // registers would cost the one-group 128^3 product an occupancy step.)
  constexpr bool kPipe = G <= 6;
  uint32_t p[S][G];
  uint32_t j = 0;
  if constexpr (kPipe) {
    load(0, p);
    for (; j + G < wm; j += G) {  // every group but the last
      uint32_t pn[S][G];
      load(j + G, pn);
      float v[S][G], xv[S][G];
      gather(p, v, xv);
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int q = 0; q < G; ++q) {
          acc[i] = fmaf(v[i][q], xv[i][q], acc[i]);
          p[i][q] = pn[i][q];
        }
    }
  } else {
    for (; j + G < wm; j += G) {  // every group but the last
      float v[S][G], xv[S][G];
      load(j, p);
      gather(p, v, xv);
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int q = 0; q < G; ++q) acc[i] = fmaf(v[i][q], xv[i][q], acc[i]);
    }
    load(j, p);
  }
  // The last group: each slice's sum is finished and stored before the next
  // slice's products wait on its gathers, so the first store is already on
  // its way while those gathers are in flight (128^3 FP16 product: 14.9 ->
  // 13.7 us in a timing copy, with the branch-free loads above).
  float v[S][G], xv[S][G];
  gather(p, v, xv);
  // Stores are not branched on: rows past n (phantom rows of the last
  // slice, slices past the end) go to row n, outside y's resource, and are
  // dropped; a branch would let the compiler sink this slice's whole group
  // into it, behind the other slice's gathers.
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int q = 0; q < G; ++q) acc[i] = fmaf(v[i][q], xv[i][q], acc[i]);
    const uint32_t t = (k0 + i) * kWave + lane;
    float r = acc[i];
    if constexpr (kFix) r = ldexpf(r, ro[i].shift(a.cd));
    const uint32_t dst = (k0 + i < a.n_slices && t < a.n) ? (IMPL ? ro[i].row() : t) : a.n;
    store_result(a.y, a.n, dst, r);
    __builtin_amdgcn_sched_barrier(0);  // keep the next slice's products after this store
  }
}

}  // namespace pksell
