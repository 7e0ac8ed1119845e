// Batched strided GEMM on CDNA4 matrix cores (FP64 and FP32 MFMA).
//
// Every contraction of the density-fitted sigma product (first-order Coulomb and
// exchange terms, the second-order amplitude strips and the amplitude-weighted
// ladder/ring contractions) and of the subspace solver is expressed as one
// GemmDesc; this file owns the only dense-contraction kernel of the library.
//
// Design (gfx950):
//  * 256 threads = 4 wave64, arranged 2x2; each wave owns a (BM/2)x(BN/2) block of
//    C made of 16x16 MFMA tiles (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).
//  * A and B tiles (BK deep) are staged through LDS in k-major layout
//    ([BK][BM+pad]) so that one MFMA operand fragment is a 16-lane contiguous
//    read; two LDS buffers and a register prefetch of the next tile overlap global
//    loads with matrix-core work (one barrier per BK step).
//  * Workgroup ids are remapped so that the tiles an XCD runs are contiguous in a
//    grouped (row-band) order: tiles sharing A rows or B columns hit the same L2.
//  * Split-K (over the flattened outer x inner reduction) writes per-split partial
//    tiles to a caller workspace; a second kernel sums them in split order, so the
//    result is deterministic and independent of the launch shape of other work.
#include "common.h"

#include <algorithm>
#include <type_traits>
#include <vector>

namespace ppw {
namespace {

template <typename T>
struct Mfma;

// Operand layout (both types): lane l supplies A[l%16][l/16] and B[l/16][l%16].
// Result layout (measured on gfx950): FP64 lane l, register r holds D[l/16 + 4r][l%16];
// FP32 lane l, register r holds D[4(l/16) + r][l%16].
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kThreads = 256;

// XCD-aware remap of a flattened workgroup id: the hardware dispatches consecutive
// ids round-robin over the 8 XCDs, so id -> (id % 8) * per + id / 8 gives each XCD a
// contiguous range of (batch, tile) work that shares operands in its own L2.
__device__ __forceinline__ long xcd_remap(long bid, long total) {
  const long per = total / 8;
  if (per > 0 && bid < per * 8) return (bid % 8) * per + bid / 8;
  return bid;
}

__device__ __forceinline__ void tile_coords(int id, int tiles_m, int tiles_n, int& tm, int& tn) {
  // grouped ordering: bands of GROUP tile-rows walked column by column
  constexpr int GROUP = 8;
  const int in_group = GROUP * tiles_n;
  const int g = id / in_group;
  const int first_m = g * GROUP;
  const int gsize = min(tiles_m - first_m, GROUP);
  const int r = id % in_group;
  tm = first_m + r % gsize;
  tn = r / gsize;
}

// ---------------------------------------------------------------------------
// FP64 tiles with both operands contiguous along k (the amplitude contraction and its
// grouped launches): operand tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: lane l of a wave writes 16 B at the wave's LDS base + 16 l),
// so no registers hold the next tile and no LDS stores are issued.  A tile row of BK = 16
// doubles is 8 slots of 16 B; (row r, pair kp) lives in slot r * 8 + (kp ^ ((r >> 1) & 7)),
// which puts the 16 rows of an MFMA fragment read in 16 different 16-byte bank groups.
// Lanes choose their source element so that each wave's 64 slots (8 rows) are filled in
// one instruction.  Ragged tiles (an edge in m, n or k, or rows not 16-byte aligned) are
// loaded through registers into the same layout.  The two LDS buffers are separate
// arrays and the loop is unrolled by two, so a buffer being filled and the buffer being
// read are distinct objects to the compiler.  MFMA operands and their order are those of
// the register-staged path, so results are bit-identical to it.
__device__ __forceinline__ int swz16(int r, int kp) { return r * 8 + (kp ^ ((r >> 1) & 7)); }

// Offset of index x along a C dimension that may be a pair (x / R, x % R) with strides
// (S, unit); R = 0 gives x * unit.  The quotient comes from a double product and one
// correction, exact for every int x.
__device__ __forceinline__ long c_index(int x, int R, long S, long unit) {
  if (R == 0) return (long)x * unit;
  int q = (int)((double)x * (1.0 / (double)R));
  int r = x - q * R;
  if (r < 0) {
    --q;
    r += R;
  } else if (r >= R) {
    ++q;
    r -= R;
  }
  return (long)q * S + (long)r * unit;
}

// Epilogue of a tile whose C rows or columns are mapped (no split-K workspace): column
// offsets once per thread, row offsets once per accumulator row.
template <typename T, typename Acc, int TM, int TN, int WTM, int WTN>
__device__ __forceinline__ void store_mapped(const GemmDesc& d, T alpha, T beta, T* __restrict__ Cb, int m0, int n0,
                                             int wm, int wn, int lane, const Acc (&acc)[TM][TN]) {
  long coff[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn * WTN + j * 16 + (lane & 15);
    coff[j] = col < d.N ? c_index(col + d.cBn, d.cRn, d.cSn, 1) : -1;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = m0 + wm * WTM + i * 16 + Mfma<T>::row(lane, r);
      if (row >= d.M) continue;
      const long ro = c_index(row, d.cRm, d.cSm, d.ldc);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (coff[j] < 0) continue;
        T* cp = Cb + ro + coff[j];
        T out = alpha * acc[i][j][r];
        if (beta != T(0)) out += beta * (*cp);
        *cp = out;
      }
    }
}

template <int BM, int BN>
__device__ __forceinline__ void gemm_tile_dma(const GemmDesc& d, double alpha, const double* __restrict__ A,
                                              const double* __restrict__ B, double beta, double* __restrict__ C,
                                              double* __restrict__ W, int splitk, long flat, int split) {
  constexpr int BK = 16;
  using acc_t = Mfma<double>::acc_t;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int SA = BM * BK, SB = BN * BK;
  constexpr int CA = BM / 32, CB = BN / 32;  // 1 KB chunks per wave (4 waves, 8 rows a chunk)
  __shared__ __attribute__((aligned(16))) double As0[SA];
  __shared__ __attribute__((aligned(16))) double As1[SA];
  __shared__ __attribute__((aligned(16))) double Bs0[SB];
  __shared__ __attribute__((aligned(16))) double Bs1[SB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const long ntiles = (long)tiles_m * tiles_n;
  const int batch = (int)(flat / ntiles);
  int tm, tn;
  tile_coords((int)(flat % ntiles), tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int b1 = batch / d.nb2, b2 = batch % d.nb2;
  const double* Atile = A + b1 * d.sA1 + b2 * d.sA2 + (long)m0 * d.lda;
  const double* Btile = B + b1 * d.sB1 + b2 * d.sB2 + (long)n0 * d.ldb;
  const int nkt = (d.K + BK - 1) / BK;
  const long total = (long)d.KB * nkt;
  const long chunk = (total + splitk - 1) / splitk;
  const long it0 = (long)split * chunk;
  const long it1 = min(total, it0 + chunk);
  const int lda32 = (int)d.lda, ldb32 = (int)d.ldb;
  const int mrem = d.M - m0, nrem = d.N - n0;
  const bool rows_ok = mrem >= BM && nrem >= BN && (d.lda % 2) == 0 && (d.ldb % 2) == 0 && (d.sAk % 2) == 0 &&
                       (d.sBk % 2) == 0 && ((uintptr_t)Atile % 16) == 0 && ((uintptr_t)Btile % 16) == 0;
  // source element (within a tile, k0 = 0) of this lane's slot in each of its chunks
  int offA[CA], offB[CB];
#pragma unroll
  for (int c = 0; c < CA; ++c) {
    const int sl = (wave + 4 * c) * 64 + lane, r = sl >> 3, kp = (sl & 7) ^ ((r >> 1) & 7);
    offA[c] = r * lda32 + 2 * kp;
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int sl = (wave + 4 * c) * 64 + lane, r = sl >> 3, kp = (sl & 7) ^ ((r >> 1) & 7);
    offB[c] = r * ldb32 + 2 * kp;
  }
  typedef double pair_t __attribute__((ext_vector_type(2)));
  // fill buffer (Ab, Bb) with the k tile (kb, kt)
  auto fill = [&](double* Ab, double* Bb, int kb, int kt) {
    const int k0 = kt * BK;
    const double* Ak = Atile + kb * d.sAk + k0;
    const double* Bk = Btile + kb * d.sBk + k0;
    const int krem = d.K - k0;
    if (rows_ok && krem >= BK) {
#pragma unroll
      for (int c = 0; c < CA; ++c)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Ak + offA[c]),
                                         (__attribute__((address_space(3))) void*)(Ab + (wave + 4 * c) * 128), 16, 0,
                                         0);
#pragma unroll
      for (int c = 0; c < CB; ++c)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Bk + offB[c]),
                                         (__attribute__((address_space(3))) void*)(Bb + (wave + 4 * c) * 128), 16, 0,
                                         0);
    } else {
      // element-wise guarded loads, zero outside the operand
#pragma unroll
      for (int i = 0; i < SA / 2 / kThreads; ++i) {
        const int pr = i * kThreads + tid, m = pr >> 3, kp = pr & 7;
        pair_t v;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kk = 2 * kp + h;
          v[h] = (m < mrem && kk < krem) ? Ak[m * lda32 + kk] : 0.0;
        }
        *reinterpret_cast<pair_t*>(Ab + 2 * swz16(m, kp)) = v;
      }
#pragma unroll
      for (int i = 0; i < SB / 2 / kThreads; ++i) {
        const int pr = i * kThreads + tid, nn = pr >> 3, kp = pr & 7;
        pair_t v;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kk = 2 * kp + h;
          v[h] = (nn < nrem && kk < krem) ? Bk[nn * ldb32 + kk] : 0.0;
        }
        *reinterpret_cast<pair_t*>(Bb + 2 * swz16(nn, kp)) = v;
      }
    }
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  auto frag = [&](const double* Ab, const double* Bb, int kk, double (&a)[TM], double (&b)[TN]) {
    const int kr = kk + (lane >> 4);
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = Ab[2 * swz16(wm * WTM + i * 16 + (lane & 15), kr >> 1) + (kr & 1)];
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = Bb[2 * swz16(wn * WTN + j * 16 + (lane & 15), kr >> 1) + (kr & 1)];
  };
  auto mma = [&](const double (&a)[TM], const double (&b)[TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<double>::mma(a[i], b[j], acc[i][j]);
  };

  if (it0 < it1) {
    int kb = (int)(it0 / nkt), kt = (int)(it0 % nkt);
    fill(As0, Bs0, kb, kt);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads into LDS have landed
    __syncthreads();
    // one k tile: prefetch the next into (An, Bn) while the MFMAs read (Ac, Bc)
    auto step = [&](const double* Ac, const double* Bc, double* An, double* Bn, long it) {
      const bool more = it + 1 < it1;
      int nkb = kb, nkt2 = kt + 1;
      if (nkt2 == nkt) {
        nkt2 = 0;
        ++nkb;
      }
      if (more) fill(An, Bn, nkb, nkt2);
      double a0[TM], b0[TN], a1[TM], b1v[TN];
      frag(Ac, Bc, 0, a0, b0);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        frag(Ac, Bc, kk + 4, a1, b1v);
        mma(a0, b0);
        if (kk + 8 < BK) frag(Ac, Bc, kk + 8, a0, b0);
        mma(a1, b1v);
      }
#pragma unroll
      for (int g = 0; g + 1 < BK / 4; ++g) {
#pragma unroll
        for (int r = 0; r < TM + TN; ++r) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        if constexpr (TM * TN > TM + TN) __builtin_amdgcn_sched_group_barrier(0x008, TM * TN - (TM + TN), 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, TM * TN, 0);
      if (more) __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
      kb = nkb;
      kt = nkt2;
    };
    for (long it = it0; it < it1; it += 2) {
      step(As0, Bs0, As1, Bs1, it);
      if (it + 1 < it1) step(As1, Bs1, As0, Bs0, it + 1);
    }
  }

  const long nbatch = (long)d.nb1 * d.nb2;
  if (!W && (d.cRm | d.cRn)) {
    store_mapped<double, acc_t, TM, TN, WTM, WTN>(d, alpha, beta, C + b1 * d.sC1 + b2 * d.sC2, m0, n0, wm, wn, lane,
                                                 acc);
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + i * 16 + Mfma<double>::row(lane, r);
        const int col = n0 + wn * WTN + j * 16 + (lane & 15);
        if (row < d.M && col < d.N) {
          const double v = acc[i][j][r];
          if (W) {
            W[((long)split * nbatch + batch) * ((long)d.M * d.N) + (long)row * d.N + col] = v;
          } else {
            double* cp = C + b1 * d.sC1 + b2 * d.sC2 + (long)row * d.ldc + col;
            double out = alpha * v;
            if (beta != 0.0) out += beta * (*cp);
            *cp = out;
          }
        }
      }
}

// LDS layouts (chosen per operand at compile time, FP64 64 banks x 4 B):
//  * operand contiguous along k in global memory (A: transA = 0, B: transB = 1):
//    tile stored [m][BK + 2]; a 16-lane group reads 16 rows at one k: bank offsets
//    36 i (+2 for the next k group) are distinct, and the global->LDS writes are
//    consecutive addresses.
//  * operand contiguous along m (or n): tile stored [k][BM + 16]; rows of 16 lanes
//    sit 32 banks apart, writes are consecutive.
// TAG only distinguishes kernel symbols (the amplitude contraction gets its own,
// so that profiles can attribute its time); the code is identical.
// One workgroup's tile of C (or, with W, of split 'split' of its reduction) for the
// flattened (batch, tile) index 'flat' of GEMM d.
// CPF (C prefetch): the C elements an accumulating tile (beta != 0, no split-K, plain
// C) will update are loaded before the reduction instead of after it, so their latency
// hides behind a short reduction; the arithmetic of the update is unchanged.
template <typename T, int BM, int BN, int BK, bool AK, bool BKC, bool CPF = false>
__device__ __forceinline__ void gemm_tile(const GemmDesc& d, T alpha, const T* __restrict__ A,
                                          const T* __restrict__ B, T beta, T* __restrict__ C, T* __restrict__ W,
                                          int splitk, long flat, int split) {
  if constexpr (std::is_same<T, double>::value && AK && BKC && BK == 16) {
    gemm_tile_dma<BM, BN>(d, alpha, A, B, beta, C, W, splitk, flat, split);
    return;
  }
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int PK = 2;   // pad of k-contiguous tiles
  constexpr int PM = 16;  // pad of m/n-contiguous tiles
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int LA = BM * BK / kThreads, LB = BN * BK / kThreads;
  static_assert(LA * kThreads == BM * BK && LB * kThreads == BN * BK, "tile/thread mismatch");
  constexpr int SA = AK ? BM * (BK + PK) : BK * (BM + PM);
  constexpr int SB = BKC ? BN * (BK + PK) : BK * (BN + PM);
  __shared__ __attribute__((aligned(16))) T As[2][SA];
  __shared__ __attribute__((aligned(16))) T Bs[2][SB];
  typedef T pair_t __attribute__((ext_vector_type(2)));
  // element (m, k) of an LDS tile
  auto aidx = [](int m, int k) { return AK ? m * (BK + PK) + k : k * (BM + PM) + m; };
  auto bidx = [](int n, int k) { return BKC ? n * (BK + PK) + k : k * (BN + PM) + n; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  const long ntiles = (long)tiles_m * tiles_n;
  const int batch = (int)(flat / ntiles);
  int tm, tn;
  tile_coords((int)(flat % ntiles), tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int b1 = batch / d.nb2, b2 = batch % d.nb2;

  const T* Ab = A + b1 * d.sA1 + b2 * d.sA2;
  const T* Bb = B + b1 * d.sB1 + b2 * d.sB2;
  const int nkt = (d.K + BK - 1) / BK;
  const long total = (long)d.KB * nkt;
  const long chunk = (total + splitk - 1) / splitk;
  const long it0 = (long)split * chunk;
  const long it1 = min(total, it0 + chunk);

  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  // Each thread moves pairs of elements that are adjacent along the contiguous
  // dimension of the operand: pair p = i * 256 + tid covers (m, k), (m, k + 1) of a
  // k-contiguous tile or (m, k), (m + 1, k) of an m-contiguous one.
  constexpr int PA = LA / 2, PB = LB / 2;
  static_assert(PA * 2 == LA && PB * 2 == LB, "pairs");
  auto a_pair = [](int p, int& m, int& k) {
    if (AK) { m = p / (BK / 2); k = 2 * (p % (BK / 2)); }
    else { m = 2 * (p % (BM / 2)); k = p / (BM / 2); }
  };
  auto b_pair = [](int p, int& n, int& k) {
    if (BKC) { n = p / (BK / 2); k = 2 * (p % (BK / 2)); }
    else { n = 2 * (p % (BN / 2)); k = p / (BN / 2); }
  };
  pair_t ra[PA], rb[PB];
  T cpre[CPF ? TM : 1][CPF ? TN : 1][4];
  if constexpr (CPF) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * WTM + i * 16 + Mfma<T>::row(lane, r);
          const int col = n0 + wn * WTN + j * 16 + (lane & 15);
          cpre[i][j][r] = (row < d.M && col < d.N) ? C[b1 * d.sC1 + b2 * d.sC2 + (long)row * d.ldc + col] : T(0);
        }
  }
  // Tile base pointers are advanced per iteration (wave-uniform 64-bit); per-element
  // offsets inside a tile are 32-bit (row * ld + k stays below 2^31 for every shape
  // the library issues), which keeps register pressure low enough for 2 waves/SIMD.
  const T* Atile = Ab + (AK ? (long)m0 * d.lda : (long)m0);
  const T* Btile = Bb + (BKC ? (long)n0 * d.ldb : (long)n0);
  const int lda32 = (int)d.lda, ldb32 = (int)d.ldb;
  // Pair loads are whole-vector loads when every pair of this tile is in range and
  // 2-element aligned (decided once per tile; wave-uniform).
  const int mrem = d.M - m0, nrem = d.N - n0;
  const bool vec_ok = mrem >= BM && nrem >= BN && (d.lda % 2) == 0 && (d.ldb % 2) == 0 && (d.sAk % 2) == 0 &&
                      (d.sBk % 2) == 0 && ((uintptr_t)Atile % (2 * sizeof(T))) == 0 &&
                      ((uintptr_t)Btile % (2 * sizeof(T))) == 0;
  auto load = [&](int kb, int kt) {
    const int k0 = kt * BK;
    const T* Ak = Atile + kb * d.sAk + (AK ? (long)k0 : (long)k0 * d.lda);
    const T* Bk = Btile + kb * d.sBk + (BKC ? (long)k0 : (long)k0 * d.ldb);
    const int krem = d.K - k0;
    if (vec_ok && krem >= BK) {
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        int m, k;
        a_pair(i * kThreads + tid, m, k);
        ra[i] = *reinterpret_cast<const pair_t*>(Ak + (AK ? (m * lda32 + k) : (k * lda32 + m)));
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        int n, k;
        b_pair(i * kThreads + tid, n, k);
        rb[i] = *reinterpret_cast<const pair_t*>(Bk + (BKC ? (n * ldb32 + k) : (k * ldb32 + n)));
      }
    } else {
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        int m, k;
        a_pair(i * kThreads + tid, m, k);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int mh = AK ? m : m + h, kh = AK ? k + h : k;
          T v = T(0);
          if (mh < mrem && kh < krem) v = Ak[AK ? (mh * lda32 + kh) : (kh * lda32 + mh)];
          ra[i][h] = v;
        }
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        int n, k;
        b_pair(i * kThreads + tid, n, k);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int nh = BKC ? n : n + h, kh = BKC ? k + h : k;
          T v = T(0);
          if (nh < nrem && kh < krem) v = Bk[BKC ? (nh * ldb32 + kh) : (kh * ldb32 + nh)];
          rb[i][h] = v;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      int m, k;
      a_pair(i * kThreads + tid, m, k);
      *reinterpret_cast<pair_t*>(&As[buf][aidx(m, k)]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      int n, k;
      b_pair(i * kThreads + tid, n, k);
      *reinterpret_cast<pair_t*>(&Bs[buf][bidx(n, k)]) = rb[i];
    }
  };
  // MFMA operand fragments of k group kk (4 deep) from LDS buffer buf
  auto frag = [&](int buf, int kk, T (&a)[TM], T (&b)[TN]) {
    const int kr = kk + (lane >> 4);
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = As[buf][aidx(wm * WTM + i * 16 + (lane & 15), kr)];
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = Bs[buf][bidx(wn * WTN + j * 16 + (lane & 15), kr)];
  };
  auto mma = [&](const T (&a)[TM], const T (&b)[TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
  };

  if (it0 < it1) {
    // (outer block, k tile) of the current iteration, stepped without division
    int kb = (int)(it0 / nkt), kt = (int)(it0 % nkt);
    load(kb, kt);
    store(0);
    __syncthreads();
    int buf = 0;
    for (long it = it0; it < it1; ++it) {
      const bool more = it + 1 < it1;
      int nkb = kb, nkt2 = kt + 1;
      if (nkt2 == nkt) {
        nkt2 = 0;
        ++nkb;
      }
      // fragments alternate between two register sets: the reads of k group g + 1
      // are in flight while the MFMAs of group g run
      T a0[TM], b0[TN], a1[TM], b1v[TN];
      frag(buf, 0, a0, b0);
      if (more) load(nkb, nkt2);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        frag(buf, kk + 4, a1, b1v);
        mma(a0, b0);
        if (kk + 8 < BK) frag(buf, kk + 8, a0, b0);
        mma(a1, b1v);
      }
      // Issue order for the scheduler: the fragment reads of each following k group
      // are spread one per MFMA over the first MFMAs of the current group, leaving
      // the rest of the group to cover their LDS latency.
#pragma unroll
      for (int g = 0; g + 1 < BK / 4; ++g) {
#pragma unroll
        for (int r = 0; r < TM + TN; ++r) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        if constexpr (TM * TN > TM + TN) __builtin_amdgcn_sched_group_barrier(0x008, TM * TN - (TM + TN), 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, TM * TN, 0);
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
      kb = nkb;
      kt = nkt2;
    }
  }

  const long nbatch = (long)d.nb1 * d.nb2;
  if (!W && (d.cRm | d.cRn)) {
    store_mapped<T, acc_t, TM, TN, WTM, WTN>(d, alpha, beta, C + b1 * d.sC1 + b2 * d.sC2, m0, n0, wm, wn, lane, acc);
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + i * 16 + Mfma<T>::row(lane, r);
        const int col = n0 + wn * WTN + j * 16 + (lane & 15);
        if (row < d.M && col < d.N) {
          const T v = acc[i][j][r];
          if (W) {
            W[((long)split * nbatch + batch) * ((long)d.M * d.N) + (long)row * d.N + col] = v;
          } else {
            T* cp = C + b1 * d.sC1 + b2 * d.sC2 + (long)row * d.ldc + col;
            T out = alpha * v;
            if constexpr (CPF) {
              out += beta * cpre[i][j][r];
            } else {
              if (beta != T(0)) out += beta * (*cp);
            }
            *cp = out;
          }
        }
      }
}

// TAG 4: the C-prefetch variant of the register-staged tile (see gemm_tile).
template <typename T, int BM, int BN, int BK, bool AK, bool BKC, int TAG>
__global__ __launch_bounds__(kThreads, 2) void gemm_kernel(GemmDesc d, T alpha, const T* __restrict__ A,
                                                        const T* __restrict__ B, T beta, T* __restrict__ C,
                                                        T* __restrict__ W, int splitk) {
  gemm_tile<T, BM, BN, BK, AK, BKC, TAG == 4>(d, alpha, A, B, beta, C, W, splitk,
                                              xcd_remap(blockIdx.x, (long)gridDim.x), blockIdx.y);
}

// Up to kGroupMax independent GEMMs of one tile shape in one grid: member g owns the
// flattened workgroup ids [start_g, start_{g+1}).  The member is found by a
// wave-uniform scan of the start table, so every member keeps the single-GEMM tile
// schedule (and the XCD remap applies over the whole grid).
constexpr int kGroupMax = 8;
template <typename T>
struct GroupMember {
  GemmDesc d;
  const T* A;
  const T* B;
  T* C;
  T alpha, beta;
  long start;
};
template <typename T>
struct GroupArgs {
  GroupMember<T> m[kGroupMax];
  int n;
};

template <typename T, int BM, int BN, int BK, bool AK, bool BKC, int TAG>
__global__ __launch_bounds__(kThreads, 2) void gemm_group_kernel(GroupArgs<T> g) {
  const long flat = xcd_remap(blockIdx.x, (long)gridDim.x);
  int j = 0;
  for (int q = 1; q < g.n; ++q)
    if (flat >= g.m[q].start) j = q;
  const GroupMember<T>& mb = g.m[__builtin_amdgcn_readfirstlane(j)];
  gemm_tile<T, BM, BN, BK, AK, BKC>(mb.d, mb.alpha, mb.A, mb.B, mb.beta, mb.C, nullptr, 1, flat - mb.start, 0);
}

template <typename T>
__global__ void splitk_reduce_kernel(GemmDesc d, T alpha, T beta, const T* __restrict__ W, T* __restrict__ C,
                                     int splitk) {
  const long per = (long)d.M * d.N;
  const long nbatch = (long)d.nb1 * d.nb2;
  const long total = per * nbatch;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
    const long batch = idx / per;
    const long rc = idx % per;
    const int row = (int)(rc / d.N), col = (int)(rc % d.N);
    T s = T(0);
    for (int k = 0; k < splitk; ++k) s += W[((long)k * nbatch + batch) * per + rc];
    const int b1 = (int)(batch / d.nb2), b2 = (int)(batch % d.nb2);
    T* cp = C + b1 * d.sC1 + b2 * d.sC2 + c_index(row, d.cRm, d.cSm, d.ldc) + c_index(d.cRn ? col + d.cBn : col, d.cRn, d.cSn, 1);
    T out = alpha * s;
    if (beta != T(0)) out += beta * (*cp);
    *cp = out;
  }
}

inline bool ntiles_total_exceeds(long n) { return n <= 0 || n > 2147483647L; }

// Workgroups of one GEMM at tile shape BM x BN (before split-K); checks the limits
// the kernel relies on.
// Reduction splits when the grid is too small to fill 256 CUs: enough for about 1024
// workgroups, at least 4 k tiles per split, within the workspace, at most 256.
int auto_splitk(long wgs, long total, size_t per, size_t ws_bytes) {
  if (wgs >= 512 || total < 8) return 1;
  long want = (1024 + wgs - 1) / wgs;
  want = std::min<long>(want, total / 4);
  if (per > 0) want = std::min<long>(want, (long)(ws_bytes / per));
  want = std::min<long>(want, 256);
  return want >= 2 ? (int)want : 1;
}

template <int BM, int BN, int BK>
long checked_workgroups(const GemmDesc& d) {
  const long nbatch = (long)d.nb1 * d.nb2;
  const long wgs = (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * nbatch;
  if (ntiles_total_exceeds(wgs)) throw InvalidArg("gemm: too many workgroups");
  // per-tile element offsets are 32-bit inside the kernel: rows of a tile that lie
  // outside the operand are never addressed, so a k-contiguous operand needs
  // min(M, BM) rows of lda, an m-contiguous one BK rows
  const double ra = d.transA == 0 ? (double)std::min(d.M, BM) * d.lda + BK : (double)BK * d.lda + BM;
  const double rb = d.transB != 0 ? (double)std::min(d.N, BN) * d.ldb + BK : (double)BK * d.ldb + BN;
  if (ra >= 2147483647.0 || rb >= 2147483647.0 || d.lda >= 2147483647L || d.ldb >= 2147483647L)
    throw InvalidArg("gemm: leading dimension too large for 32-bit tile offsets");
  if (d.cRm < 0 || d.cRn < 0) throw InvalidArg("gemm: negative C index split");
  return wgs;
}

constexpr long kCUs = 256;
constexpr long kResident = 512;  // workgroups resident at once: 256 CUs x 2

template <typename T, int BM, int BN, int BK, bool AK, bool BKC, int TAG>
void launch(const GemmDesc& d, T alpha, const T* A, const T* B, T beta, T* C, hipStream_t s, Workspace ws) {
  const int tiles_m = (d.M + BM - 1) / BM, tiles_n = (d.N + BN - 1) / BN;
  const long nbatch = (long)d.nb1 * d.nb2;
  checked_workgroups<BM, BN, BK>(d);
  const long ntiles = (long)tiles_m * tiles_n;
  // Wave quantisation: when the last of several waves of 128 x 128 tiles would run at
  // most half full, the trailing tile columns that make up that wave are peeled off and
  // computed with 64 x 64 tiles (four times the workgroups, a quarter of the work each),
  // so the tail takes about a quarter of a tile's time.  Every output element is
  // accumulated over the same sequence of MFMA k steps in both tile shapes, so the result
  // is bit-identical to the unpeeled GEMM.  The peeled part has its own kernel symbol
  // (TAG + 2) so that traces tell the two apart.
  if constexpr (TAG < 2 && BM == 128 && BN == 128) {
   if (nbatch == 1 && ntiles >= 2 * kResident && d.splitk <= 1) {
    const long rem = ntiles % kResident;
    const int cols = (int)((rem + tiles_m - 1) / tiles_m);
    if (rem > 0 && rem <= kResident / 2 && cols < tiles_n) {
      const int nmain = (tiles_n - cols) * BN;
      GemmDesc dm = d, dr = d;
      dm.N = nmain;
      dr.N = d.N - nmain;
      launch<T, BM, BN, BK, AK, BKC, TAG>(dm, alpha, A, B, beta, C, s, Workspace{});
      const T* Br = B + (BKC ? (long)nmain * d.ldb : (long)nmain);
      T* Cr = C + nmain;
      if (d.cRn) {  // mapped columns: the tail maps its columns from nmain on
        dr.cBn = d.cBn + nmain;
        Cr = C;
      }
      launch<T, BM / 2, BN / 2, BK, AK, BKC, TAG + 2>(dr, alpha, A, Br, beta, Cr, s, Workspace{});
      return;
    }
   }
  }
  const int nkt = (d.K + BK - 1) / BK;
  const long total = (long)d.KB * nkt;
  const size_t per = (size_t)d.M * d.N * nbatch * sizeof(T);
  int splitk = auto_splitk(ntiles * nbatch, total, per, ws.bytes);
  if (d.splitk > 0) {
    splitk = d.splitk;
    if (splitk > 1 && (splitk > 256 || ws.bytes / per < (size_t)splitk))
      throw InvalidArg("gemm: workspace too small for the requested reduction splits");
  }
  dim3 grid((unsigned)(ntiles * nbatch), (unsigned)splitk, 1);
  if constexpr (TAG == 0 && BM == 64 && !(std::is_same<T, double>::value && AK && BKC)) {
    // short accumulating reductions: load C before the reduction (same arithmetic)
    if (splitk == 1 && beta != T(0) && total <= 4 && !(d.cRm | d.cRn)) {
      gemm_kernel<T, BM, BN, BK, AK, BKC, 4><<<grid, kThreads, 0, s>>>(d, alpha, A, B, beta, C, nullptr, 1);
      PPW_LAUNCH_CHECK();
      return;
    }
  }
  if (splitk == 1) {
    gemm_kernel<T, BM, BN, BK, AK, BKC, TAG><<<grid, kThreads, 0, s>>>(d, alpha, A, B, beta, C, nullptr, 1);
    PPW_LAUNCH_CHECK();
  } else {
    T* W = static_cast<T*>(ws.ptr);
    gemm_kernel<T, BM, BN, BK, AK, BKC, TAG><<<grid, kThreads, 0, s>>>(d, alpha, A, B, beta, C, W, splitk);
    PPW_LAUNCH_CHECK();
    const long n = (long)d.M * d.N * nbatch;
    const int blocks = (int)std::min<long>((n + 255) / 256, 8192);
    splitk_reduce_kernel<T><<<blocks, 256, 0, s>>>(d, alpha, beta, W, C, splitk);
    PPW_LAUNCH_CHECK();
  }
}

template <typename T, int TAG = 0>
void gemm_dispatch(const GemmDesc& d, T alpha, const T* A, const T* B, T beta, T* C, hipStream_t s,
                   Workspace ws) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  if (d.K <= 0 || d.KB <= 0) throw InvalidArg("gemm: empty reduction");
  const bool big = d.M >= 96 && d.N >= 96 && d.tile != 64;
  const bool ak = d.transA == 0, bk = d.transB != 0;
#define PPW_GEMM_CASE(BMv, BNv, AKv, BKv)                                           \
  if (ak == AKv && bk == BKv) {                                                     \
    launch<T, BMv, BNv, 16, AKv, BKv, TAG>(d, alpha, A, B, beta, C, s, ws);         \
    return;                                                                         \
  }
  if (big) {
    PPW_GEMM_CASE(128, 128, true, true)
    PPW_GEMM_CASE(128, 128, true, false)
    PPW_GEMM_CASE(128, 128, false, true)
    PPW_GEMM_CASE(128, 128, false, false)
  } else {
    PPW_GEMM_CASE(64, 64, true, true)
    PPW_GEMM_CASE(64, 64, true, false)
    PPW_GEMM_CASE(64, 64, false, true)
    PPW_GEMM_CASE(64, 64, false, false)
  }
#undef PPW_GEMM_CASE
}

// One grouped launch of n <= kGroupMax members sharing the tile shape.
template <typename T, int BM, int BN, int BK, bool AK, bool BKC, int TAG>
void launch_group(const GemmCall<T>* const* calls, int n, hipStream_t s) {
  GroupArgs<T> g{};
  long total = 0;
  for (int i = 0; i < n; ++i) {
    const GemmCall<T>& c = *calls[i];
    g.m[i] = GroupMember<T>{c.d, c.A, c.B, c.C, c.alpha, c.beta, total};
    total += checked_workgroups<BM, BN, BK>(c.d);
  }
  g.n = n;
  if (ntiles_total_exceeds(total)) throw InvalidArg("gemm: too many workgroups in a group");
  gemm_group_kernel<T, BM, BN, BK, AK, BKC, TAG><<<dim3((unsigned)total), kThreads, 0, s>>>(g);
  PPW_LAUNCH_CHECK();
}

template <typename T, int TAG>
void group_dispatch(bool big, bool ak, bool bk, const GemmCall<T>* const* calls, int n, hipStream_t s) {
#define PPW_GROUP_CASE(BMv, BNv, AKv, BKv)                              \
  if (ak == AKv && bk == BKv) {                                         \
    launch_group<T, BMv, BNv, 16, AKv, BKv, TAG>(calls, n, s);          \
    return;                                                             \
  }
  if (big) {
    PPW_GROUP_CASE(128, 128, true, true)
    PPW_GROUP_CASE(128, 128, true, false)
    PPW_GROUP_CASE(128, 128, false, true)
    PPW_GROUP_CASE(128, 128, false, false)
  } else {
    PPW_GROUP_CASE(64, 64, true, true)
    PPW_GROUP_CASE(64, 64, true, false)
    PPW_GROUP_CASE(64, 64, false, true)
    PPW_GROUP_CASE(64, 64, false, false)
  }
#undef PPW_GROUP_CASE
}

template <typename T>
void single_dispatch(const GemmCall<T>& c, hipStream_t s) {
  if (c.tag >= 2) {
    if constexpr (std::is_same<T, float>::value)
      gemm_sbf16(c.d, c.alpha, c.A, c.B, c.beta, c.C, s, c.tag == 3);
    else
      throw InvalidArg("split-BF16 products take FP32 operands");
    return;
  }
  if (c.tag == 1)
    gemm_dispatch<T, 1>(c.d, c.alpha, c.A, c.B, c.beta, c.C, s, c.ws);
  else
    gemm_dispatch<T, 0>(c.d, c.alpha, c.A, c.B, c.beta, c.C, s, c.ws);
}

// Independent GEMMs issued together: members with the same tile shape (and symbol
// tag) go into grouped launches when together they fill the chip without split-K;
// the rest (a lone member, or a set too small to fill 256 CUs) are launched one by
// one, where split-K applies.
template <typename T>
int gemm_group_impl(const std::vector<GemmCall<T>>& calls, hipStream_t s) {
  int grouped = 0;
  struct Key {
    bool big, ak, bk;
    int tag;
    bool operator==(const Key& o) const { return big == o.big && ak == o.ak && bk == o.bk && tag == o.tag; }
  };
  std::vector<Key> keys;
  std::vector<std::vector<const GemmCall<T>*>> sets;
  for (const auto& c : calls) {
    const GemmDesc& d = c.d;
    if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) continue;
    if (d.K <= 0 || d.KB <= 0) throw InvalidArg("gemm: empty reduction");
    if (d.splitk > 1 || c.tag >= 2) {
      // fixed reduction splits need the split-K launch; split-BF16 has its own kernel
      single_dispatch(c, s);
      continue;
    }
    const Key k{d.M >= 96 && d.N >= 96 && d.tile != 64, d.transA == 0, d.transB != 0, c.tag};
    size_t i = 0;
    while (i < keys.size() && !(keys[i] == k)) ++i;
    if (i == keys.size()) {
      keys.push_back(k);
      sets.emplace_back();
    }
    sets[i].push_back(&c);
  }
  for (size_t i = 0; i < keys.size(); ++i) {
    const Key& k = keys[i];
    auto& set = sets[i];
    long wgs = 0;
    for (auto* c : set)
      wgs += k.big ? checked_workgroups<128, 128, 16>(c->d) : checked_workgroups<64, 64, 16>(c->d);
    if (set.size() == 1 || wgs < 512) {
      for (auto* c : set) single_dispatch(*c, s);
      continue;
    }
    for (size_t j = 0; j < set.size(); j += kGroupMax) {
      const int n = (int)std::min<size_t>(kGroupMax, set.size() - j);
      if (k.tag == 1)
        group_dispatch<T, 1>(k.big, k.ak, k.bk, set.data() + j, n, s);
      else
        group_dispatch<T, 0>(k.big, k.ak, k.bk, set.data() + j, n, s);
      ++grouped;
    }
  }
  return grouped;
}

// ---------------------------------------------------------------------------
// Split-BF16 products.  An FP32 value x is carried as hi = bf16(x) (round to nearest
// even) and lo = bf16(x - hi); a b is taken as hi_a lo_b + lo_a hi_b + hi_a hi_b with FP32
// accumulation (the dropped lo_a lo_b and the rounding of lo leave about 2^-16 of |a b|
// per product).  Operands are split once, in memory, before the product (split_sbf16):
// a row of values is a sequence of 32-byte chunks, chunk c holding the bf16 hi parts of
// values 8c .. 8c+7 and then their 8 lo parts.  A value still occupies 4 bytes, so rows
// keep their FP32 strides (a multiple of 8 values) and an FP32 array is split in place.
//
// Kernel: WM x WN wave64s on BM x BN tiles (4 x 2 on 256 x 256 at one workgroup per CU,
// 2 x 2 on 128 x 128 or 64 x 64 at two), ST LDS stages; a k tile is 32 values = 4 chunks
// = 128 B per row, loaded straight into LDS (global_load_lds_dwordx4) in the swizzled
// slot layout of the FP64 kernel (16-byte slot s of row r at 8r + (s ^ ((r >> 1) & 7)),
// logical slot 2c holding chunk c's hi parts and 2c + 1 its lo parts), so a fragment
// read of 16 rows x 16 B touches every bank once and no conversion happens in the loop.
// Each wave computes 32 x 32 blocks with v_mfma_f32_32x32x16_bf16 (on gfx950 it issues
// at twice the rate of the 16x16x32 form: 2.0 against 1.1 PFLOP/s measured with
// register-only chains), three MFMAs per block and 16-value k step: lane l supplies row
// l % 32 and chunk l / 32 of the step; block results: lane l, register r holds row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.  Ragged tiles (an edge in m, n or k) are
// copied chunk by chunk through registers into the same layout; values past K inside the
// last chunk of a row must be zero (split_sbf16 of a zero-padded row leaves them so).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int kSbBK = 32;

__device__ __forceinline__ int row32(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// WM x WN waves (64 WM WN threads), each owning a (BM / WM) x (BN / WN) block of the tile;
// ST LDS buffers, the loads of tile kt + ST - 1 issued while tile kt is multiplied; OCC
// workgroups per CU (register budget).  TAG only distinguishes kernel symbols (1: the
// amplitude contraction, so that profiles can attribute its time); the code is identical.
template <int BM, int BN, int WM, int WN, int ST, int OCC, int TAG = 0>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm_sbf16_kernel(
    GemmDesc d, float alpha, const float* __restrict__ A, const float* __restrict__ B, float beta,
    float* __restrict__ C) {
  constexpr int BK = kSbBK, NW = WM * WN, NT = 64 * NW;
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 32, TN = WTN / 32;
  constexpr int SA = BM * BK, SB = BN * BK;       // storage floats per buffer
  constexpr int CA = BM / (8 * NW), CB = BN / (8 * NW);  // 1 KB wave loads (8 rows each) per operand tile
  static_assert(CA * 8 * NW == BM && CB * 8 * NW == BN && TM * 32 == WTM && TN * 32 == WTN, "tile shape");
  static_assert(ST >= 2 && ST <= 4 && (ST - 2) * (CA + CB) <= 63, "stages");
  __shared__ __attribute__((aligned(16))) float As[ST][SA];
  __shared__ __attribute__((aligned(16))) float Bs[ST][SB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave / WN, wn = wave % WN;
  const int tiles_m = (d.M + BM - 1) / BM, tiles_n = (d.N + BN - 1) / BN;
  int tm, tn;
  tile_coords((int)xcd_remap(blockIdx.x, (long)gridDim.x), tiles_m, tiles_n, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const float* At = A + (long)m0 * d.lda;
  const float* Bt = B + (long)n0 * d.ldb;
  const int lda32 = (int)d.lda, ldb32 = (int)d.ldb;
  const int mrem = d.M - m0, nrem = d.N - n0;
  const bool rows_ok = mrem >= BM && nrem >= BN;
  int offA[CA], offB[CB];
#pragma unroll
  for (int c = 0; c < CA; ++c) {
    const int sl = (wave + NW * c) * 64 + lane, r = sl >> 3, sg = (sl & 7) ^ ((r >> 1) & 7);
    offA[c] = r * lda32 + 4 * sg;
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int sl = (wave + NW * c) * 64 + lane, r = sl >> 3, sg = (sl & 7) ^ ((r >> 1) & 7);
    offB[c] = r * ldb32 + 4 * sg;
  }
  // tiles loaded straight into LDS: all of them when the tile is whole in m and n, except
  // a ragged last k tile
  const int nkt = (d.K + BK - 1) / BK;
  const int ndma = rows_ok ? d.K / BK : 0;
  auto fill = [&](int buf, int kt) {
    const int k0 = kt * BK;
    const float* Ak = At + k0;
    const float* Bk = Bt + k0;
    float* Ab = As[buf];
    float* Bb = Bs[buf];
    if (kt < ndma) {
#pragma unroll
      for (int c = 0; c < CA; ++c)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Ak + offA[c]),
                                         (__attribute__((address_space(3))) void*)(Ab + (wave + NW * c) * 256), 16, 0,
                                         0);
#pragma unroll
      for (int c = 0; c < CB; ++c)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(Bk + offB[c]),
                                         (__attribute__((address_space(3))) void*)(Bb + (wave + NW * c) * 256), 16, 0,
                                         0);
    } else {
#pragma unroll
      for (int i = 0; i < SA / 4 / NT; ++i) {
        const int q = i * NT + tid, r = q >> 3, sg = q & 7;
        f32x4_t v = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if (r < mrem && k0 + 8 * (sg >> 1) < d.K) v = *reinterpret_cast<const f32x4_t*>(Ak + r * lda32 + 4 * sg);
        *reinterpret_cast<f32x4_t*>(Ab + 4 * swz16(r, sg)) = v;
      }
#pragma unroll
      for (int i = 0; i < SB / 4 / NT; ++i) {
        const int q = i * NT + tid, r = q >> 3, sg = q & 7;
        f32x4_t v = f32x4_t{0.f, 0.f, 0.f, 0.f};
        if (r < nrem && k0 + 8 * (sg >> 1) < d.K) v = *reinterpret_cast<const f32x4_t*>(Bk + r * ldb32 + 4 * sg);
        *reinterpret_cast<f32x4_t*>(Bb + 4 * swz16(r, sg)) = v;
      }
    }
  };
  f32x16_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  const int rl = lane & 31, hl = lane >> 5;
  // one k tile = two 16-value steps: the fragment reads of both steps are issued first
  // (B, then A in MFMA order), so the second step's reads land during the first step's
  // MFMAs
  auto tile = [&](int buf) {
    const float* Ab = As[buf];
    const float* Bb = Bs[buf];
    bf16x8_t ah[2][TM], al[2][TM], bh[2][TN], bl[2][TN];
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      const int ch = 2 * st + hl;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm * WTM + i * 32 + rl;
        ah[st][i] = *reinterpret_cast<const bf16x8_t*>(Ab + 4 * swz16(r, 2 * ch));
        al[st][i] = *reinterpret_cast<const bf16x8_t*>(Ab + 4 * swz16(r, 2 * ch + 1));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = wn * WTN + j * 32 + rl;
        bh[st][j] = *reinterpret_cast<const bf16x8_t*>(Bb + 4 * swz16(r, 2 * ch));
        bl[st][j] = *reinterpret_cast<const bf16x8_t*>(Bb + 4 * swz16(r, 2 * ch + 1));
      }
    }
    // per step and column block: the hi-lo products of its row blocks, then lo-hi, then
    // hi-hi (consecutive MFMAs accumulate into different blocks, each element still sums
    // hl, lh, hh in that order, and a column block's B fragments die once it is done)
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[st][i], bl[st][j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[st][i], bh[st][j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[st][i], bh[st][j], acc[i][j], 0, 0, 0);
      }
    // issue order pinned: the first step's fragment reads, then its MFMAs with the second
    // step's reads interleaved one by one, then the second step's MFMAs
    constexpr int R = 2 * (TM + TN), Mf = 3 * TM * TN, P = R < Mf ? R : Mf;
    __builtin_amdgcn_sched_group_barrier(0x100, R, 0);
#pragma unroll
    for (int n = 0; n < P; ++n) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    if constexpr (Mf > P) __builtin_amdgcn_sched_group_barrier(0x008, Mf - P, 0);
    if constexpr (R > P) __builtin_amdgcn_sched_group_barrier(0x100, R - P, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, Mf, 0);
  };
  // vmcnt(n), other counters left alone (gfx9 s_waitcnt encoding)
  constexpr int kWaitKeep = 0x0F70 | (((ST - 2) * (CA + CB)) & 15) | (((((ST - 2) * (CA + CB)) >> 4) & 3) << 14);
#pragma unroll
  for (int s0 = 0; s0 + 1 < ST; ++s0)
    if (s0 < nkt) fill(s0, s0);
  if (ST > 2 && ST - 1 <= ndma)  // tile 0 has landed
    __builtin_amdgcn_s_waitcnt(kWaitKeep);
  else
    __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < nkt; ++kt) {
    const int kn = kt + ST - 1;
    if (kn < nkt) fill(buf == 0 ? ST - 1 : buf - 1, kn);
    tile(buf);
    // tile kt + 1 must have landed for every wave: the loads of the tiles after it may stay
    // in flight when they all went straight into LDS
    if (kt + 1 < nkt) {
      if (ST > 2 && kt + ST - 1 < ndma)
        __builtin_amdgcn_s_waitcnt(kWaitKeep);
      else
        __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    __syncthreads();
    buf = buf + 1 == ST ? 0 : buf + 1;
  }
  // epilogue: column offsets once per thread, row offsets once per accumulator row
  const bool mapped = (d.cRm | d.cRn) != 0;
  long coff[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = n0 + wn * WTN + j * 32 + rl;
    coff[j] = col < d.N ? (mapped ? c_index(col + d.cBn, d.cRn, d.cSn, 1) : (long)col) : -1;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + wm * WTM + i * 32 + row32(lane, r);
      if (row >= d.M) continue;
      const long ro = mapped ? c_index(row, d.cRm, d.cSm, d.ldc) : (long)row * d.ldc;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (coff[j] < 0) continue;
        float* cp = C + ro + coff[j];
        float out = alpha * acc[i][j][r];
        if (beta != 0.0f) out += beta * (*cp);
        *cp = out;
      }
    }
}

// In-place split of n / 8 chunks of 8 FP32 values into the chunk layout above.
__global__ void split_sbf16_kernel(long nchunks, float* __restrict__ x) {
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < nchunks; c += (long)gridDim.x * blockDim.x) {
    f32x4_t* p = reinterpret_cast<f32x4_t*>(x + 8 * c);
    const f32x4_t a = p[0], b = p[1];
    bf16x8_t hi, lo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      hi[t] = (__bf16)a[t];
      hi[t + 4] = (__bf16)b[t];
      lo[t] = (__bf16)(a[t] - (float)hi[t]);
      lo[t + 4] = (__bf16)(b[t] - (float)hi[t + 4]);
    }
    *reinterpret_cast<bf16x8_t*>(x + 8 * c) = hi;
    *reinterpret_cast<bf16x8_t*>(x + 8 * c + 4) = lo;
  }
}

}  // namespace

int gemm_auto_splitk(const GemmDesc& d, size_t ws_bytes, bool fp32) {
  if (d.splitk > 0) return d.splitk;
  const bool big = d.M >= 96 && d.N >= 96 && d.tile != 64;
  const int BM = big ? 128 : 64, BN = BM;
  const long ntiles = (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  const long nbatch = (long)d.nb1 * d.nb2;
  const long total = (long)d.KB * ((d.K + 15) / 16);
  const size_t per = (size_t)d.M * d.N * nbatch * (fp32 ? sizeof(float) : sizeof(double));
  return auto_splitk(ntiles * nbatch, total, per, ws_bytes);
}

void gemm_sbf16(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C, hipStream_t s,
                bool amplitude) {
  if (d.M <= 0 || d.N <= 0) return;
  if (d.K <= 0) throw InvalidArg("gemm: empty reduction");
  if (d.transA != 0 || d.transB == 0 || d.KB != 1 || d.nb1 != 1 || d.nb2 != 1)
    throw InvalidArg("split-BF16 GEMM: operands contiguous along k, no batch or outer reduction");
  if (d.lda % 8 || d.ldb % 8 || d.lda < d.K || d.ldb < d.K || (uintptr_t)A % 16 || (uintptr_t)B % 16)
    throw InvalidArg("split-BF16 GEMM: operand rows must start on 32-byte chunks (leading dimensions a multiple "
                     "of 8 values and at least K, 16-byte aligned operands)");
  if (d.M >= 96 && d.N >= 96) {
    // 256 x 256 tiles (8 waves of 64 x 128, one workgroup per CU: 453 TF/s measured on a
    // 8192 x 65536 x 32768 product) against 128 x 128 (4 waves of 64 x 64, two per CU:
    // 386 TF/s): each round of resident 256-tiles holds twice the work of a round of
    // 128-tiles and runs about 1.05 times faster per flop, so the larger tile is taken
    // when its whole rounds finish first
    const long t256 = (long)((d.M + 255) / 256) * ((d.N + 255) / 256);
    const long t128 = (long)((d.M + 127) / 128) * ((d.N + 127) / 128);
    const double r256 = (double)((t256 + kCUs - 1) / kCUs), r128 = (double)((t128 + 2 * kCUs - 1) / (2 * kCUs));
    if (d.tile == 256 || (d.tile != 128 && r256 * 2.0 / 1.05 < r128)) {
      const long wgs = checked_workgroups<256, 256, kSbBK>(d);
      if (amplitude)
        gemm_sbf16_kernel<256, 256, 4, 2, 2, 1, 1><<<dim3((unsigned)wgs), 512, 0, s>>>(d, alpha, A, B, beta, C);
      else
        gemm_sbf16_kernel<256, 256, 4, 2, 2, 1><<<dim3((unsigned)wgs), 512, 0, s>>>(d, alpha, A, B, beta, C);
    } else {
      const long wgs = checked_workgroups<128, 128, kSbBK>(d);
      if (amplitude)
        gemm_sbf16_kernel<128, 128, 2, 2, 2, 2, 1><<<dim3((unsigned)wgs), kThreads, 0, s>>>(d, alpha, A, B, beta, C);
      else
        gemm_sbf16_kernel<128, 128, 2, 2, 2, 2><<<dim3((unsigned)wgs), kThreads, 0, s>>>(d, alpha, A, B, beta, C);
    }
  } else {
    const long wgs = checked_workgroups<64, 64, kSbBK>(d);
    gemm_sbf16_kernel<64, 64, 2, 2, 2, 2><<<dim3((unsigned)wgs), kThreads, 0, s>>>(d, alpha, A, B, beta, C);
  }
  PPW_LAUNCH_CHECK();
}

void split_sbf16(long n, float* x, hipStream_t s) {
  if (n <= 0) return;
  if (n % 8 || (uintptr_t)x % 16) throw InvalidArg("split_sbf16: a whole number of 8-value chunks, 16-byte aligned");
  const long chunks = n / 8;
  const int blocks = (int)std::max<long>(1, std::min<long>((chunks + 255) / 256, 65536));
  split_sbf16_kernel<<<blocks, 256, 0, s>>>(chunks, x);
  PPW_LAUNCH_CHECK();
}

int gemm_group_f64(const std::vector<GemmCall<double>>& calls, hipStream_t s) { return gemm_group_impl(calls, s); }
int gemm_group_f32(const std::vector<GemmCall<float>>& calls, hipStream_t s) { return gemm_group_impl(calls, s); }

void gemm_f64(const GemmDesc& d, double alpha, const double* A, const double* B, double beta, double* C,
              hipStream_t s, Workspace ws) {
  gemm_dispatch<double>(d, alpha, A, B, beta, C, s, ws);
}

void gemm_f64_hhat(const GemmDesc& d, double alpha, const double* A, const double* B, double beta, double* C,
                   hipStream_t s, Workspace ws) {
  gemm_dispatch<double, 1>(d, alpha, A, B, beta, C, s, ws);
}

void gemm_f32_hhat(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C,
                   hipStream_t s, Workspace ws) {
  gemm_dispatch<float, 1>(d, alpha, A, B, beta, C, s, ws);
}

void gemm_f32(const GemmDesc& d, float alpha, const float* A, const float* B, float beta, float* C,
              hipStream_t s, Workspace ws) {
  gemm_dispatch<float>(d, alpha, A, B, beta, C, s, ws);
}

}  // namespace ppw
