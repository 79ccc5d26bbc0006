// Workgroup-level building blocks of the setup and of the lambda path:
//   * Gram tiles on f32 MFMA (128 x 128 output tile, 256 threads: 4 waves in
//     2 x 2) and on bf16 MFMA at float32 accuracy (the six products of a
//     three-way bf16 split, 512 threads: 8 waves in 4 x 2),
//   * the general f32 MFMA tile product of the lambda path (128 x 128, 512
//     threads: 8 waves in 2 x 4),
//   * float64 64 x 64 block products on f64 MFMA (256 threads),
//   * the diagonal-block Cholesky / triangular inverse, panel solve, trailing
//     update, blocked inverse steps and the K^{-1} = L^{-T} L^{-1} product.
// The single-problem setup launches one workgroup per tile; the grouped
// (batched) launches run the same functions over the tiles of every problem.
#pragma once

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "mfma.hpp"

namespace pogs {

constexpr int NB = 64;        // Cholesky block size
constexpr int LSF = NB + 2;   // row stride of the float64 LDS stages

constexpr int KCF = 64;       // k depth of one float64 block-product stage
struct F64Stage {             // 67.6 KB
  double a[KCF][LSF];
  double b[KCF][LSF];
};
struct CholLds {              // 66.6 KB
  double L[NB][NB + 1];
  double X[NB][NB + 1];
};
constexpr int kGramTB = 128;  // f32 Gram tile
constexpr int kGramKC = 16;   // k depth of one f32 stage
struct GramStage {            // 18.4 KB (row stride 144: the 16-lane row groups of an MFMA operand read land on disjoint banks)
  float a[kGramKC][kGramTB + 16];
  float b[kGramKC][kGramTB + 16];
};

constexpr int kGemmKC = 16;   // k depth of one stage of the general f32 tile product (32 measured the same)
struct GemmStage {            // 18.4 KB (row stride 144, as GramStage)
  float a[kGemmKC][kGramTB + 16];
  float b[kGemmKC][kGramTB + 16];
};

// Tile pair t of a lower triangle (ti >= tj), row by row.
__device__ inline void tri_index(int t, int *ti, int *tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *ti = i;
  *tj = t - i * (i + 1) / 2;
}

typedef float GramAcc __attribute__((ext_vector_type(4)));

// Gram tile (ti, tj) over k in [k0, k1): TALL: sum_k A[k][i] A[k][j] (A^T A),
// else sum_k A[i][k] A[j][k] (A A^T).  Each wave owns a 64 x 64 quarter as
// 4 x 4 f32 MFMA 16x16x4 blocks; out(row, col, value) visits the tile's
// elements (tile-local indices).  Reads beyond m / n are zero.  k0 is a
// multiple of kGramKC.  Stages of kGramKC k in two LDS buffers: the next
// stage is loaded into registers while the MFMAs of the current one run and
// stored into the other buffer after them (one barrier per stage).  Ends
// with a barrier.
template <bool TALL, class Out>
__device__ void gram_tile_f32(const float *__restrict__ A, int m, int n, int ld, int ti, int tj, int k0, int k1,
                              GramStage (&st)[2], Out out) {
  constexpr int TB = kGramTB, KC = kGramKC;
  constexpr int NL = KC * TB / 4 / 256;  // float4 loads per thread per panel
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool diag = ti == tj;
  typedef float f4 __attribute__((ext_vector_type(4)));
  GramAcc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = GramAcc{0.f, 0.f, 0.f, 0.f};
  f4 ra[NL], rb[NL];
  auto load = [&](int kk0) {
#pragma unroll
    for (int h = 0; h < NL; ++h) {
      const int f = t + h * 256;
      ra[h] = f4{0.f, 0.f, 0.f, 0.f};
      rb[h] = f4{0.f, 0.f, 0.f, 0.f};
      if (TALL) {
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k;
        if (row < k1) {
          const int ca = ti * TB + c, cb = tj * TB + c;
          if (ca < n) ra[h] = *reinterpret_cast<const f4 *>(A + (size_t)row * ld + ca);
          if (!diag && cb < n) rb[h] = *reinterpret_cast<const f4 *>(A + (size_t)row * ld + cb);
        }
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int kc = kk0 + kq;  // kc + 3 < ld (kk0 % 16 == 0, ld % 64 == 0, kk0 < n <= ld)
        const int rra = ti * TB + r, rrb = tj * TB + r;
        if (rra < m) ra[h] = *reinterpret_cast<const f4 *>(A + (size_t)rra * ld + kc);
        if (!diag && rrb < m) rb[h] = *reinterpret_cast<const f4 *>(A + (size_t)rrb * ld + kc);
      }
    }
  };
  auto store = [&](GramStage &sd, int kk0) {
#pragma unroll
    for (int h = 0; h < NL; ++h) {
      const int f = t + h * 256;
      if (TALL) {
        const int k = f >> 5, c = (f & 31) * 4;
        *reinterpret_cast<f4 *>(&sd.a[k][c]) = ra[h];
        if (!diag) *reinterpret_cast<f4 *>(&sd.b[k][c]) = rb[h];
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int kc = kk0 + kq;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool ok = kc + u < k1;
          sd.a[kq + u][r] = ok ? ra[h][u] : 0.f;
          if (!diag) sd.b[kq + u][r] = ok ? rb[h][u] : 0.f;
        }
      }
    }
  };
  load(k0);
  store(st[0], k0);
  __syncthreads();
  int cur = 0;
  for (int kk0 = k0; kk0 < k1; kk0 += KC) {
    const bool more = kk0 + KC < k1;
    if (more) load(kk0 + KC);
    const GramStage &sc = st[cur];
    const float(*pb)[TB + 16] = diag ? sc.a : sc.b;
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float av[4], bv[4];
      const int kr = k4 + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        av[b] = sc.a[kr][wi * 64 + b * 16 + cl];
        bv[b] = pb[kr][wj * 64 + b * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(st[cur ^ 1], kk0 + KC);
    __syncthreads();
    cur ^= 1;
  }
  // f32 16x16x4 result layout: lane l, element r -> row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out(wi * 64 + i * 16 + 4 * (lane >> 4) + r, wj * 64 + j * 16 + (lane & 15), acc[i][j][r]);
}

// Gram tile of a tall matrix from bf16 MFMAs at float32 accuracy.  Every
// float32 entry x is split into three bf16 pieces, x = h + m + l (h = bf16(x),
// m = bf16(x - h), l = bf16(x - h - m), each rounded to nearest; the
// remainders are exact in float32, so the three pieces hold all 24 bits of x
// outside the subnormal range), and a product x y is formed from the six
// products of pieces whose weight is at least 2^-16 of h h:
// l h + h l + m m + m h + h m + h h (the three dropped ones are below 2^-24 of
// x y, the size of a float32 product's rounding).  Each bf16 product is exact
// in the float32 accumulator of the MFMA, so the tile carries the errors of
// float32 accumulation only, at six bf16 MFMAs per product of float32 values
// (MI355X: 2.5 PFLOP/s bf16 against 157 TFLOP/s float32).  The h h products
// and the five smaller ones go to separate accumulators, added at the end:
// with all six in one, every 16 rows put six roundings of the large partial
// sum into it, and over a 4000-row split that cost the 20000 x 2000
// projection a factor of six in accuracy (1.1e-6 against the FP64 projection,
// 1.7e-7 with two accumulators, 2.3e-7 with the float32-MFMA Gram; 9.7e-8 with
// two accumulators and the 2900-row splits of two dispatch rounds).
// The tile is sum_k A[k][i] A[k][j] over k in [k0, k1), tile (ti, tj); k0 is
// a multiple of kG6KC; columns >= n and rows >= k1 read as zero.
// Stages of kG6KC rows: the loads of the stage after next go out before a
// stage's MFMAs, and the next stage's pieces are stored into the other LDS
// buffer after them (one barrier per stage).  512 threads (8 waves), each
// wave a 32 x 64 part of the tile.  Ends with a barrier.
constexpr int kG6KC = 16;  // k depth of one stage (one MFMA depth)
// [operand][piece][column][k]: 24 KB per stage.  A column's 16 k are two 16-byte
// halves, swapped in columns c with bit 3 of c set, so the 16 lanes of a
// 16-byte access (16 consecutive columns, one half) hit 16 disjoint bank
// groups.
struct Gram6Stage {
  __bf16 v[2][3][kGramTB][kG6KC];
};
__device__ inline int g6_half(int c, int h) { return (h ^ ((c >> 3) & 1)) * 8; }
typedef float Gram6Acc __attribute__((ext_vector_type(16)));

template <class Out>
__device__ void gram_tile_bf16x6(const float *__restrict__ A, int n, int ld, int ti, int tj, int k0, int k1,
                                 Gram6Stage (&st)[2], Out out) {
  typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
  constexpr int TB = kGramTB;
  // 8 waves: wave w owns rows 32 (w / 2) .. + 31 and columns 64 (w % 2) .. + 63
  // of the tile, as 1 x 2 MFMA 32x32x16 blocks
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool diag = ti == tj;
  // staging: thread t takes column t % 128 and rows 4 (t / 128) .. + 3 of a
  // stage; a row is wave-uniform, so each load is a uniform row base plus
  // the lane's column (columns and rows past the ends are clamped, then
  // zeroed)
  constexpr int E = 4;
  const int sc = t & (TB - 1), sh = __builtin_amdgcn_readfirstlane((t >> 7) * E);
  const int ca = ti * TB + sc, cb = tj * TB + sc;
  const bool oka = ca < n, okb = !diag && cb < n;
  const int cla = min(ca, n - 1), clb = diag ? cla : min(cb, n - 1);
  const int sk = g6_half(sc, sh >> 3) + (sh & 7);  // where this thread's E k go in its column
  // two register sets: the loads of stage s + 2 go out while stage s is
  // multiplied and stage s + 1 waits in the other set for its store
  float ra[2][E], rb[2][E];
  // loads only (no wait): rows and columns past the ends are zeroed when the
  // stage is stored
  auto load = [&](auto set, int kk0) {
    constexpr int S = decltype(set)::value;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float *rp = A + (size_t)min(kk0 + sh + e, k1 - 1) * ld;
      ra[S][e] = rp[cla];
      rb[S][e] = rp[clb];  // unused on a diagonal tile (clb = cla there)
    }
  };
  // x = h + m + l by pairs: v_cvt_pk_bf16_f32 rounds two values to nearest
  // and packs them; a packed pair widens back by a shift and a mask
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  auto widen = [](unsigned pk) { return f2{__uint_as_float(pk << 16), __uint_as_float(pk & 0xffff0000u)}; };
  auto pack = [](f2 v) { return __builtin_bit_cast(unsigned, __builtin_convertvector(v, b2)); };
  auto split_store = [&](const float (&r)[E], bool ok, int kk0, __bf16 (*dst)[kGramTB][kG6KC]) {
    u2 ph, pm, pl;
#pragma unroll
    for (int q = 0; q < E / 2; ++q) {
      const int row = kk0 + sh + 2 * q;
      const f2 x = {ok && row < k1 ? r[2 * q] : 0.f, ok && row + 1 < k1 ? r[2 * q + 1] : 0.f};
      const unsigned h = pack(x);
      const f2 r1 = x - widen(h);
      const unsigned mm = pack(r1);
      const f2 r2 = r1 - widen(mm);
      ph[q] = h;
      pm[q] = mm;
      pl[q] = pack(r2);
    }
    *reinterpret_cast<u2 *>(&dst[0][sc][sk]) = ph;
    *reinterpret_cast<u2 *>(&dst[1][sc][sk]) = pm;
    *reinterpret_cast<u2 *>(&dst[2][sc][sk]) = pl;
  };
  auto store = [&](Gram6Stage &sd, auto set, int kk0) {
    constexpr int S = decltype(set)::value;
    split_store(ra[S], oka, kk0, sd.v[0]);
    if (!diag) split_store(rb[S], okb, kk0, sd.v[1]);
  };
  // the h h products accumulate in acc, the five smaller ones in acs: the
  // large accumulator then takes one rounding per 16 rows instead of six
  Gram6Acc acc[2], acs[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = acs[j][r] = 0.f;
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  // loads are issued whether or not their stage exists (rows clamp to
  // k1 - 1): a conditional load makes the compiler wait for every load in
  // flight where the paths join
  load(S0{}, k0);
  load(S1{}, k0 + kG6KC);
  store(st[0], S0{}, k0);
  __syncthreads();
  int cur = 0;
  // MFMA 32x32x16 operands: lane l holds 8 consecutive k (8 (l / 32) ..) of
  // row (A) or column (B) l % 32
  const int fr = lane & 31;
  // (bit 3 of a column index is that of fr: multiples of 32 leave it alone)
  const int fka = g6_half(wi * 32 + fr, lane >> 5), fkb = g6_half(wj * 64 + fr, lane >> 5);
  const int ob = diag ? 0 : 1;
  // stage kk0 is in LDS buffer cur, stage kk0 + kG6KC in register set S
  auto step = [&](int kk0, auto set) {
    constexpr int S = decltype(set)::value;
    load(std::integral_constant<int, 1 - S>{}, kk0 + 2 * kG6KC);
    const Gram6Stage &sc_ = st[cur];
    bf8 a[3], b[2][3];
#pragma unroll
    for (int pc = 0; pc < 3; ++pc) {
      a[pc] = *reinterpret_cast<const bf8 *>(&sc_.v[0][pc][wi * 32 + fr][fka]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j][pc] = *reinterpret_cast<const bf8 *>(&sc_.v[ob][pc][wj * 64 + j * 32 + fr][fkb]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      Gram6Acc c = acs[j];
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[j][0], c, 0, 0, 0);  // l h
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][2], c, 0, 0, 0);  // h l
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][1], c, 0, 0, 0);  // m m
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][0], c, 0, 0, 0);  // m h
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][1], c, 0, 0, 0);  // h m
      acs[j] = c;
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][0], acc[j], 0, 0, 0);  // h h
    }
    // the other buffer was last read before the previous barrier
    store(st[cur ^ 1], set, kk0 + kG6KC);
    __syncthreads();
    cur ^= 1;
  };
  // stages in pairs, with no condition in the loop (a stage past k1 is all
  // zeros and adds nothing)
  for (int kk0 = k0; kk0 < k1; kk0 += 2 * kG6KC) {
    step(kk0, S1{});
    step(kk0 + kG6KC, S0{});
  }
  // 32x32 result layout: lane l, element r -> row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      out(wi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), wj * 64 + j * 32 + (lane & 31), acc[j][r] + acs[j][r]);
}

// General f32 MFMA tile product: tile (i0.., j0..) of sum_{k in [k0, k1)} opA(i, k) B(k, j)
// with opA(i, k) = A[k * lda + i] (A_T: A stored K x M) or A[i * lda + k]
// (A stored M x K), B stored K x N row-major (ldb % 4 == 0).  Rows >= M,
// columns >= N and k >= k1 read as zero; lda and ldb are multiples of 4 and
// the rows of A and B are readable up to the next multiple of 16 elements
// past M (A_T), k1 (not A_T) and N.  out(row, col, value) gets tile-local
// indices.  128 x 128 tile, kGemmKC-deep stages, 512 threads: 8 waves in 2 (rows) x 4 (columns),
// each 64 x 32 as 4 x 2 f32 MFMA 16x16x4 blocks, so that every SIMD holds two
// waves and one wave's LDS reads and stage wait run under the other's MFMAs.
template <bool A_T, class Out>
__device__ void gemm_tile_f32(const float *__restrict__ A, int lda, int M, const float *__restrict__ B, int ldb,
                              int N, int i0, int j0, int k0, int k1, GemmStage (&st)[2], Out out) {
  constexpr int KC = kGemmKC, NH = KC / 16;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wi = w >> 2, wj = w & 3;
  typedef float f4 __attribute__((ext_vector_type(4)));
  GramAcc acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = GramAcc{0.f, 0.f, 0.f, 0.f};
  // stage k range [kk0, kk0 + KC) into registers (KC / 16 float4 of A and
  // of B per thread), then into an LDS buffer; the next stage's loads are in
  // flight while the MFMAs of the current one run
  f4 ra[NH], rb[NH];
  auto load = [&](int kk0) {
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int f = t + h * 512;  // float4 index in a KC x 128 stage
      {                           // B: rows kk0 + k, columns j0 + c .. c + 3
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k, col = j0 + c;
        rb[h] = f4{0.f, 0.f, 0.f, 0.f};
        if (row < k1 && col < N) rb[h] = *reinterpret_cast<const f4 *>(B + (size_t)row * ldb + col);
      }
      ra[h] = f4{0.f, 0.f, 0.f, 0.f};
      if (A_T) {
        const int k = f >> 5, c = (f & 31) * 4;
        const int row = kk0 + k, col = i0 + c;
        if (row < k1 && col < M) ra[h] = *reinterpret_cast<const f4 *>(A + (size_t)row * lda + col);
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int row = i0 + r, kc = kk0 + kq;
        if (row < M && kc < k1) ra[h] = *reinterpret_cast<const f4 *>(A + (size_t)row * lda + kc);
      }
    }
  };
  auto store = [&](GemmStage &sd, int kk0) {
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int f = t + h * 512;
      {
        const int k = f >> 5, c = (f & 31) * 4;
        *reinterpret_cast<f4 *>(&sd.b[k][c]) = rb[h];
      }
      if (A_T) {
        const int k = f >> 5, c = (f & 31) * 4;
        *reinterpret_cast<f4 *>(&sd.a[k][c]) = ra[h];
      } else {
        const int r = f & 127, kq = (f >> 7) * 4;
        const int kc = kk0 + kq;
#pragma unroll
        for (int u = 0; u < 4; ++u) sd.a[kq + u][r] = kc + u < k1 ? ra[h][u] : 0.f;
      }
    }
  };
  load(k0);
  store(st[0], k0);
  __syncthreads();
  int cur = 0;
  for (int kk0 = k0; kk0 < k1; kk0 += KC) {
    const bool more = kk0 + KC < k1;
    if (more) load(kk0 + KC);
    const GemmStage &sc = st[cur];
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      float av[4], bv[2];
      const int kr = k4 + (lane >> 4), cl = lane & 15;
#pragma unroll
      for (int b = 0; b < 4; ++b) av[b] = sc.a[kr][wi * 64 + b * 16 + cl];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sc.b[kr][wj * 32 + b * 16 + cl];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) store(st[cur ^ 1], kk0 + KC);
    __syncthreads();
    cur ^= 1;
  }
  // 16x16 result layout: lane l, element r -> row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out(wi * 64 + i * 16 + 4 * (lane >> 4) + r, wj * 32 + j * 16 + (lane & 15), acc[i][j][r]);
}

// One 64 (k) x 64 (index) chunk of op(k, x) = p[k * sk + x * sx], with
// either sx == 1 (contiguous along x) or sk == 1 (contiguous along k), as
// eight 16-byte loads per thread (every base address and stride is even).
struct F64Chunk {
  double2 v[8];
};

__device__ inline void chunk_load(F64Chunk &c, const double *p, int64_t sk, int64_t sx) {
  const int t = threadIdx.x;
  const int outer = t >> 5, pr = (t & 31) * 2;
  if (sx == 1) {
#pragma unroll
    for (int r = 0; r < 8; ++r) c.v[r] = *reinterpret_cast<const double2 *>(p + (int64_t)(outer + 8 * r) * sk + pr);
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) c.v[r] = *reinterpret_cast<const double2 *>(p + (int64_t)(outer + 8 * r) * sx + pr);
  }
}

// Store a loaded chunk k-major: s[k][x].
__device__ inline void chunk_store(const F64Chunk &c, double (*s)[LSF], bool xcontig) {
  const int t = threadIdx.x;
  const int outer = t >> 5, pr = (t & 31) * 2;
  if (xcontig) {
#pragma unroll
    for (int r = 0; r < 8; ++r) *reinterpret_cast<double2 *>(&s[outer + 8 * r][pr]) = c.v[r];
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      s[pr][outer + 8 * r] = c.v[r].x;
      s[pr + 1][outer + 8 * r] = c.v[r].y;
    }
  }
}

// acc += sum_{k < K} opA(i, k) opB(k, j) for a 64 x 64 float64 tile, with
// opA(i, k) = pa[i * sai + k * sak], opB(k, j) = pb[k * sbk + j * sbj],
// each operand contiguous along one of its two indices, K a multiple of 64.
// Stages of 64 k; the next stage is loaded into registers while the MFMAs
// of the current one run.  Ends with a barrier: the stages may be reused and
// the operands overwritten afterwards.
__device__ inline void block_product(F64Acc acc[2][2], const double *pa, int64_t sai, int64_t sak, const double *pb,
                                     int64_t sbk, int64_t sbj, int K, F64Stage &st) {
  const int w = threadIdx.x >> 6;
  const int wi = w >> 1, wj = w & 1;
  const bool a_icontig = sai == 1, b_jcontig = sbj == 1;
  F64Chunk ca, cb;
  chunk_load(ca, pa, sak, sai);
  chunk_load(cb, pb, sbk, sbj);
  for (int k0 = 0; k0 < K; k0 += KCF) {
    if (k0) __syncthreads();
    chunk_store(ca, st.a, a_icontig);
    chunk_store(cb, st.b, b_jcontig);
    __syncthreads();
    if (k0 + KCF < K) {
      chunk_load(ca, pa + (int64_t)(k0 + KCF) * sak, sak, sai);
      chunk_load(cb, pb + (int64_t)(k0 + KCF) * sbk, sbk, sbj);
    }
#pragma unroll
    for (int k4 = 0; k4 < KCF; k4 += 4) f64_tile_step<LSF>(acc, st.a, st.b, k4, wi * 32, wj * 32);
  }
  __syncthreads();
}

__device__ inline void acc_zero(F64Acc acc[2][2]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f64acc_zero();
}

template <class Fn> __device__ inline void acc_store(const F64Acc acc[2][2], Fn fn) {
  const int w = threadIdx.x >> 6;
  f64_tile_store(acc, (w >> 1) * 32, (w & 1) * 32, fn);
}

// sqrt(p) and 1 / sqrt(p) for p > 0 by Goldschmidt's coupled iteration
// (g -> sqrt(p), h -> 1 / (2 sqrt(p)); e = 1/2 - g h, then g += g e and
// h += h e), started from the hardware reciprocal square root estimate.
// Each step squares the relative error, so two steps take the estimate's
// ~2^-22 to the float64 rounding level.  The two updates of a step are
// independent, so the dependent chain is one multiply and two fmas per step,
// shorter on the factor's critical path than sqrt() and a division, which
// are correctly rounded expansions.
__device__ inline void sqrt_rsqrt(double p, double &g, double &rs) {
  const double y = __builtin_amdgcn_rsq(p);
  g = p * y;
  double h = 0.5 * y;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
  }
  rs = 2.0 * h;
}

// Value of v in lane K of each row of 16 lanes, for every lane of that row:
// one 64-bit DPP move (row_newbcast is the DPP control gfx950 allows on 64-bit
// moves), no scalar registers.  Every lane reads a valid source lane, so the
// old value (with bound_ctrl set) is never used.
template <int K> __device__ inline double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xf, 0xf, true);
}

// 16 x 16 leaf, one copy per row of 16 lanes: lane r holds row r of the
// block in a[0..15] and column r of W = L^{-1} in x[0..15].  Column J of the
// Cholesky factor: L_JJ = sqrt(piv) (lane J), L_rJ = a_J / sqrt(piv), then
// the right-looking update a_I -= L_rJ L_IJ of the later columns.  Step J of
// W's forward substitution by columns needs exactly column J of L and
// 1 / L_JJ, which every lane holds at that point (the broadcasts are shared):
// x_J = acc_J / L_JJ, then acc_I -= L_IJ x_J (acc starts as column r of I).
// The pivots of I + G are at least 1 in exact arithmetic; one that is not
// positive and finite is counted in nbad (the setup then fails), off the
// dependent chain.
template <int I>
__device__ inline void leaf_pair(double (&a)[16], double (&acc)[16], double lj, double xj) {
  const double l = row_bcast<I>(lj);  // L_IJ
  a[I] = fma(-lj, l, a[I]);
  acc[I] = fma(-l, xj, acc[I]);
}
template <int J, int... K>
__device__ inline void leaf_updates(double (&a)[16], double (&acc)[16], double lj, double xj,
                                    std::integer_sequence<int, K...>) {
  (leaf_pair<J + 1 + K>(a, acc, lj, xj), ...);
}
template <int J>
__device__ inline void leaf_column(double (&a)[16], double (&acc)[16], double (&x)[16], unsigned &nbad, int r) {
  const double piv = row_bcast<J>(a[J]);
  nbad += (piv > 0.0 && isfinite(piv)) ? 0u : 1u;
  double g, rd;
  sqrt_rsqrt(piv, g, rd);
  const double lj = r == J ? g : a[J] * rd;
  a[J] = lj;
  x[J] = acc[J] * rd;
  leaf_updates<J>(a, acc, lj, x[J], std::make_integer_sequence<int, 15 - J>{});
}
template <int... J>
__device__ inline void leaf_factor_inverse(double (&a)[16], double (&x)[16], unsigned &nbad, int r,
                                           std::integer_sequence<int, J...>) {
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = r == k ? 1.0 : 0.0;
  (leaf_column<J>(a, acc, x, nbad, r), ...);
  // An empty statement that every lane executes and that reads the results:
  // without it the compiler moves the leaf into the branch where only some
  // lanes store it, and that schedule holds over 300 registers instead of ~110.
#pragma unroll
  for (int k = 0; k < 16; ++k) asm volatile("" ::"v"(a[k]), "v"(x[k]));
}

// Value of v in lane l (l uniform), as two 32-bit lane reads.
__device__ inline double lane_bcast(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// acc += sum_{k < 16} a(i, k) b(k, j) for one 16 x 16 block (one wave,
// f64 MFMA 16x16x4); result element r of lane l is (4 r + l / 16, l % 16).
template <class FA, class FB> __device__ inline F64Acc mfma_block16(F64Acc acc, FA a, FB b) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int k4 = 0; k4 < 16; k4 += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(i, k4 + kq), b(k4 + kq, i), acc, 0, 0, 0);
  return acc;
}

// Factor diagonal block kb of K (Q x Q, row-major, lower part used) and
// invert the factor, in LDS with the whole workgroup (4 waves).  The 64 x 64
// block is factored recursively over 16 x 16 sub-blocks s = 0..3:
//   leaf:   L_ss = chol(B_ss) and W_s = L_ss^{-1}, in the registers of every
//           row of 16 lanes (row r of L_ss and column r of W_s in lane r % 16;
//           the values other rows need are DPP row broadcasts), no LDS round
//           trips inside the 16-step chains;
//   panel:  L_rs = B_rs W_s^T for the row blocks r > s (f64 MFMA, one wave per block);
//   update: B_IJ -= L_Is L_Js^T for s < J <= I (f64 MFMA).
// Then X = L^{-1} by block diagonals: X_ii = W_i, and for i > j
// X_ij = -W_i sum_{j <= k < i} L_ik X_kj, the partial sums parked in the
// (unused) upper blocks of X.  potrf_diag_core works on the block in s.L
// (only its lower triangle, diagonal included, is read) and leaves L in the
// lower blocks of s.L and X in the lower blocks of s.X; potrf_diag loads
// block kb of K first and afterwards writes L_kk (upper part zeroed) back into
// K and L_kk^{-1} into Dinv block kb.  A pivot that is not positive and finite
// counts in *bad.  Launched with 256 threads.
__device__ __forceinline__ void potrf_diag_core(CholLds &s, unsigned *bad) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  unsigned nbad = 0;
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int s0 = sb * 16;
    // leaf (every row of 16 lanes of every wave computes the same values)
    double a[16], x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = s.L[s0 + r16][s0 + k];
    leaf_factor_inverse(a, x, nbad, r16, std::make_integer_sequence<int, 16>{});
    if (lane < 16) {  // every wave holds the leaf: wave w writes columns 4w .. 4w + 3
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if ((k >> 2) == w) {
          s.L[s0 + lane][s0 + k] = a[k];
          s.X[s0 + k][s0 + lane] = x[k];
        }
    }
    __syncthreads();
    // panel
    const int nrb = 3 - sb;
    if (w < nrb) {
      const int rb = (sb + 1 + w) * 16;
      F64Acc acc = mfma_block16(
          f64acc_zero(), [&](int i, int k) { return s.L[rb + i][s0 + k]; },
          [&](int k, int j) { return s.X[s0 + j][s0 + k]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) s.L[rb + 4 * r + q4][s0 + r16] = acc[r];
    }
    __syncthreads();
    // trailing update of the lower blocks
    const int ntr = nrb * (nrb + 1) / 2;
    for (int b = w; b < ntr; b += 4) {
      const int ii = b >= 3 ? 2 : (b >= 1 ? 1 : 0);
      const int I = (sb + 1 + ii) * 16, J = (sb + 1 + b - ii * (ii + 1) / 2) * 16;
      F64Acc acc = mfma_block16(
          f64acc_zero(), [&](int i, int k) { return s.L[I + i][s0 + k]; },
          [&](int k, int j) { return s.L[J + j][s0 + k]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) s.L[I + 4 * r + q4][J + r16] -= acc[r];
    }
    __syncthreads();
  }
  // X = L^{-1}: block diagonal d = i - j, pairs (i, j) one per wave
  for (int d = 1; d < 4; ++d) {
    const bool mine = w < 4 - d;
    const int i = (d + w) * 16, j = w * 16;
    if (mine) {
      F64Acc acc = f64acc_zero();
      for (int k = j; k < i; k += 16)
        acc = mfma_block16(
            acc, [&](int ii, int kk) { return s.L[i + ii][k + kk]; },
            [&](int kk, int jj) { return s.X[k + kk][j + jj]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) s.X[j + 4 * r + q4][i + r16] = acc[r];  // T_ij, parked in block (j, i)
    }
    __syncthreads();
    if (mine) {
      F64Acc acc = mfma_block16(
          f64acc_zero(), [&](int ii, int kk) { return s.X[i + ii][i + kk]; },
          [&](int kk, int jj) { return s.X[j + kk][i + jj]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) s.X[i + 4 * r + q4][j + r16] = -acc[r];
    }
    __syncthreads();
  }
  if (nbad && t == 0) atomicAdd(bad, nbad);
}

__device__ __forceinline__ void potrf_diag(double *K, int Q, int kb, double *Dinv, unsigned *bad, CholLds &s) {
  const int t = threadIdx.x;
  double *blk = K + (size_t)kb * NB * Q + (size_t)kb * NB;
  // every load in flight before the first LDS store (256 threads)
  constexpr int kPer = NB * NB / 256;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + 256 * u;
    v[u] = blk[(size_t)(e / NB) * Q + e % NB];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + 256 * u;
    s.L[e / NB][e % NB] = v[u];
  }
  __syncthreads();
  potrf_diag_core(s, bad);
  double *dv = Dinv + (size_t)kb * NB * NB;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + 256 * u;
    const int r = e / NB, c = e % NB;
    blk[(size_t)r * Q + c] = c <= r ? s.L[r][c] : 0.0;
    dv[e] = (c >> 4) > (r >> 4) ? 0.0 : s.X[r][c];
  }
  __syncthreads();
}

// L_ib,kb = K_ib,kb L_kb,kb^{-T}   (in place)
__device__ inline void trsm_tile(double *K, int Q, int kb, int ib, const double *Dinv, F64Stage &st) {
  double *blk = K + (size_t)ib * NB * Q + (size_t)kb * NB;
  const double *dv = Dinv + (size_t)kb * NB * NB;
  F64Acc acc[2][2];
  acc_zero(acc);
  block_product(acc, blk, Q, 1, dv, 1, NB, NB, st);
  acc_store(acc, [&](int r, int c, double v) { blk[(size_t)r * Q + c] = v; });
}

// K_I,J -= L_I,kb L_J,kb^T
__device__ inline void syrk_tile(double *K, int Q, int kb, int I, int J, F64Stage &st) {
  const double *LI = K + (size_t)I * NB * Q + (size_t)kb * NB;
  const double *LJ = K + (size_t)J * NB * Q + (size_t)kb * NB;
  double *C = K + (size_t)I * NB * Q + (size_t)J * NB;
  F64Acc acc[2][2];
  acc_zero(acc);
  block_product(acc, LI, Q, 1, LJ, 1, Q, NB, st);
  acc_store(acc, [&](int r, int c, double v) { C[(size_t)r * Q + c] -= v; });
}

// Blocked L^{-1} by right-looking block forward substitution of L X = I:
// X holds B = I - sum_{k<i} L_.k X_k. (initialised to the identity); step i
// sets X_ij = L_ii^{-1} B_ij for j <= i (trtri_scale_tile), then
// B_rj -= L_ri X_ij for r > i, j <= i (trtri_update_tile).  Every launch of a
// step is many independent 64 x 64 x 64 products.
__device__ inline void trtri_scale_tile(const double *Dinv, double *X, int Q, int i, int j, F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  double *C = X + (size_t)i * NB * Q + (size_t)j * NB;
  block_product(acc, Dinv + (size_t)i * NB * NB, NB, 1, C, Q, 1, NB, st);
  acc_store(acc, [&](int r, int c, double v) { C[(size_t)r * Q + c] = v; });
}

__device__ inline void trtri_update_tile(const double *K, double *X, int Q, int i, int r, int j, F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *pa = K + (size_t)r * NB * Q + (size_t)i * NB;  // L_ri
  const double *pb = X + (size_t)i * NB * Q + (size_t)j * NB;  // X_ij
  block_product(acc, pa, Q, 1, pb, Q, 1, NB, st);
  double *C = X + (size_t)r * NB * Q + (size_t)j * NB;
  acc_store(acc, [&](int rr, int cc, double v) { C[(size_t)rr * Q + cc] -= v; });
}

// X <- I on the lower block triangle, diagonal blocks included whole (the
// block products read full 64 x 64 blocks; blocks above the diagonal are
// never read).
__device__ inline void trtri_init_rows(double *X, int Q, int row0, int row1) {
  for (int i = row0; i < row1; ++i) {
    const int jend = (i / NB + 1) * NB;
    for (int j = threadIdx.x; j < jend; j += blockDim.x) X[(size_t)i * Q + j] = i == j ? 1.0 : 0.0;
  }
}

// K^{-1}_I,J = sum_{k >= I} X_k,I^T X_k,J for I >= J, written and mirrored as T
// (entries of index >= q skipped).
template <typename T>
__device__ inline void kinv_tile(const double *X, int Q, int nbt, int q, T *Kinv, int ldk, int I, int J,
                                 F64Stage &st) {
  F64Acc acc[2][2];
  acc_zero(acc);
  const double *pa = X + (size_t)I * NB * Q + (size_t)I * NB;
  const double *pb = X + (size_t)I * NB * Q + (size_t)J * NB;
  block_product(acc, pa, 1, Q, pb, Q, 1, (nbt - I) * NB, st);
  acc_store(acc, [&](int r, int c, double v) {
    const int gi = I * NB + r, gj = J * NB + c;
    if (gi < q && gj < q) {
      Kinv[(size_t)gi * ldk + gj] = (T)v;
      Kinv[(size_t)gj * ldk + gi] = (T)v;
    }
  });
}

}  // namespace pogs
