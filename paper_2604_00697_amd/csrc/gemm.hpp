// Tiled MFMA GEMM for gfx950 in "NT" form:
//     C[i][j] = sum_k A[i][k] * Bt[j][k]
// with both operands stored k-contiguous in the MFMA operand type, in
// zero-padded buffers (rows padded to the tile, k padded to the k-step).
// Producers write their outputs in the layout the next product consumes
// (plain or transposed), which removes all transposes from the inner loops.
//
// Data path per workgroup (NT = 64 * WGM * WGN threads):
//   global --(global_load_lds_dwordx4: 16 bytes per lane straight into LDS)-->
//   S-stage LDS ring, each staged row 128 bytes with its 16-byte chunks
//   XOR-swizzled by (row % 8) so the fragment reads of 16 rows spread over the
//   banks --> 16x16 MFMA fragments, double-buffered in registers (the next
//   k-tile is read while the second half of this one's MFMAs issue)
//   --> fp32 accumulators --> fp32 tile staged in LDS --> epilogue functor.
// Up to S-1 k-tiles are in flight per workgroup; each wave waits only for its
// own loads of the next k-tile (vmcnt) before the workgroup barrier.
// Triangular operands skip their zero k-blocks through the tile schedule.
#pragma once
#include <hip/hip_ext.h>

#include "common.hpp"

#define LDS_AS __attribute__((address_space(3)))

// A64: fp32 operands accumulated on the fp64 matrix cores (the tile is
// rounded to fp32 once, when it is staged for the epilogue).
template <int BM_, int BN_, int WGM_, int WGN_, typename T_, int S_, bool A64_ = false>
struct Cfg {
  using T = T_;
  static constexpr int BM = BM_, BN = BN_, WGM = WGM_, WGN = WGN_, S = S_;
  static constexpr bool A64 = A64_;
  static_assert(!A64 || std::is_same<T_, float>::value, "fp64 accumulation takes fp32 operands");
  using Acc = typename std::conditional<A64_, f64x4, f32x4>::type;
  static constexpr int NW = WGM * WGN, NT = 64 * NW;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int TM = WM / 16, TN = WN / 16;
  static constexpr int KPL = 16 / (int)sizeof(T);   // operand elements per 16-byte chunk
  static constexpr int BK = 8 * KPL;                // k per stage: 8 chunks = 128 bytes per row
  static constexpr int ROWB = 128;                  // LDS bytes of one staged row
  static constexpr int STAGE = (BM + BN) * ROWB;    // LDS bytes of one stage
  static constexpr int IPW = (BM + BN) / (8 * NW);  // 1 KB load instructions per wave per stage
  static constexpr int LDC = BN + 1;                // epilogue staging row, floats
  static constexpr int SMEM_MAIN = S * STAGE;
  // epilogue: staged tile + 16*NT bytes of reduction scratch (+ extra per epilogue)
  static constexpr int SMEM_EPI = (BM * LDC + 4 * NT) * (int)sizeof(float);
  static constexpr int smem(int extra) {
    return SMEM_MAIN > SMEM_EPI + extra ? SMEM_MAIN : SMEM_EPI + extra;
  }
  static_assert(WM % 16 == 0 && WN % 16 == 0, "wave tile must be a multiple of 16");
  static_assert((BM + BN) % (8 * NW) == 0 && BM % 8 == 0,
                "each wave loads whole 8-row groups");
  static_assert(S >= 2, "at least two stages");
  static_assert(IPW * (S - 1) <= 63, "outstanding loads must fit the vmcnt counter");
  static_assert(SMEM_MAIN <= 160 * 1024, "LDS capacity");
};

// One operand: k-contiguous rows of length >= the padded k extent.
template <typename T>
struct Opnd {
  const T *p;
  long ld;
};

// ------------------------------------------------------------------ schedule
enum : int { K_LO_M0 = 1, K_LO_N0 = 2, K_HI_M1 = 4, K_HI_N1 = 8 };

// Maps a workgroup index b (blockIdx.x) to an output tile and its k-range.
//   sym = 0: rectangular grid of mt x nt tiles;
//   sym = 1: lower-triangular tiles (I >= J) of an mt x mt grid.
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2), so block b is renumbered to run consecutive tiles on one XCD; for
// rectangular grids consecutive tiles share a column block (I fastest), so an
// XCD streams one slice of the B operand against the whole A operand.
// rule: K_* bounds (k >= m0, k >= n0, k < m0+BM, k < n0+BN) skipping blocks of
// a triangular operand known to be zero.  nsplit > 1 splits the k-range into
// BK-aligned pieces (split-K) selected by blockIdx.y.  skip (optional): a
// device flag; when it is set, every tile skips its k-loop (zero accumulators)
// and only the epilogue runs.
struct Sched {
  int mt, nt, sym, nsplit, K, rule;
  const int *skip;
  long gs;  // grouped launch: bytes between the problems' workspaces (0: one problem)
  // b: the workgroup's index among the tiles
  template <class C>
  IFS_DEV void tile(int b, int &m0, int &n0, int &kb, int &ke, int &ti) const {
    const int ntile = sym ? mt * (mt + 1) / 2 : mt * nt;
    // XCD-contiguous renumbering: blocks b, b+8, b+16, ... share XCD b % 8
    const int per = (ntile + 7) / 8, rem = ntile % 8;
    const int x = b % 8, q = b / 8;
    int t;
    if (rem == 0 || x < rem) t = x * per + q;
    else t = rem * per + (x - rem) * (per - 1) + q;
    // k-ranges bounded above by the row or column block (a lower-triangular
    // operand) grow with I (and J <= I): such tiles run longest first, so the
    // launch does not end on a long tile started last.  ti stays the tile's
    // position in the canonical order, which indexes per-tile partials.
    int I, J;
    if (sym) {
      if ((rule & (K_HI_M1 | K_HI_N1)) && !(rule & (K_LO_M0 | K_LO_N0))) t = ntile - 1 - t;
      I = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      while (I * (I + 1) / 2 > t) --I;
      J = t - I * (I + 1) / 2;
      ti = t;
    } else {
      J = t / mt;
      I = t - J * mt;
      if (rule & K_HI_M1) I = mt - 1 - I;
      ti = J * mt + I;
    }
    m0 = I * C::BM;
    n0 = J * C::BN;
    int lo = 0, hi = K;
    if (rule & K_LO_M0) lo = max(lo, m0);
    if (rule & K_LO_N0) lo = max(lo, n0);
    if (rule & K_HI_M1) hi = min(hi, m0 + C::BM);
    if (rule & K_HI_N1) hi = min(hi, n0 + C::BN);
    lo = (lo / C::BK) * C::BK;
    if (nsplit > 1) {
      const int nkt = hi > lo ? (hi - lo + C::BK - 1) / C::BK : 0;
      const int per_s = (nkt + nsplit - 1) / nsplit;
      const int s = blockIdx.y;
      kb = lo + s * per_s * C::BK;
      ke = min(hi, lo + (s + 1) * per_s * C::BK);
    } else {
      kb = lo;
      ke = hi;
    }
  }
};

struct TileInfo {
  int m0, n0, ti, split;
};

// s_waitcnt with vmcnt = v and lgkmcnt = 0 (gfx9 encoding; expcnt left open).
template <int v>
IFS_DEV void wait_vm_lgkm0() {
  static_assert(v >= 0 && v <= 63, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((v & 15) | (7 << 4) | (0 << 8) | ((v >> 4) << 14));
}
// Wait until at most n stages (of IPW loads each) of this wave are in flight.
template <int IPW, int NMAX>
IFS_DEV void wait_stages(int n) {
  if constexpr (NMAX > 0) {
    if (n >= NMAX) {
      wait_vm_lgkm0<NMAX * IPW>();
      return;
    }
    wait_stages<IPW, NMAX - 1>(n);
  } else {
    wait_vm_lgkm0<0>();
  }
}

// Epilogues declaring kRegs = true take the accumulators in registers
// (run_regs: acc[i][j][q] = C[WM wm + 16 i + 4 (lane/16) + q][WN wn + 16 j + lane % 16],
// or for fp64 accumulators (A64) row WM wm + 16 i + 4 q + lane/16; LDS free for
// their own use); the others get the tile staged in LDS (run).
template <class E, class = void>
struct EpiTakesRegs : std::false_type {};
template <class E>
struct EpiTakesRegs<E, std::void_t<decltype(E::kRegs)>> : std::bool_constant<E::kRegs> {};

template <int v>
struct IC {
  static constexpr int value = v;
};

// ------------------------------------------------------------------ generated B operand
// NoGen: both operands are loaded from global memory.
// Side role of a product's launch: nside workgroups after the tiles form
// a = L^T m~ (one wave per row, from the fp32 transpose Lt of the same L, m~
// from the call's arguments); they start as the short tiles of a triangular
// product finish, so the matrix-vector product runs beside the product's tail
// instead of after it.
struct SideRows {
  const float *Lt;
  long ldl;
  const CallArgs *ca;
  float *a;
  int M, nside;
  IFS_DEV void shift(long o) {
    Lt = gsh(Lt, o); ca = gsh(ca, o); a = gsh(a, o);
  }
  IFS_DEV void run(int blk) const {
    const int row = blk * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (row >= M) return;
    const float s = row_dot(Lt + (long)row * ldl, ca->m, nullptr, M);
    if ((threadIdx.x & 63) == 0) a[row] = s;
  }
};

struct NoGen {
  static constexpr bool kOn = false, kSide = false;
  int side_blocks() const { return 0; }
  IFS_DEV void side(int) const {}
  IFS_DEV void shift(long) {}
  template <class C>
  struct State {
    IFS_DEV void init(const NoGen &, int, int) {}
    IFS_DEV void prefetch(int) {}
    IFS_DEV void gen(unsigned char *, int) {}
  };
};

// A loaded B operand with the side role.
struct SideOnly : NoGen {
  static constexpr bool kSide = true;
  SideRows rows;
  int side_blocks() const { return rows.nside; }
  IFS_DEV void side(int blk) const { rows.run(blk); }
  IFS_DEV void shift(long o) { rows.shift(o); }
};

// KufGen: the B operand of V = L^T K_uf is the kernel-matrix tile
//   Bt[n][m] = K_uf[m][n] = sf2 exp(-1/2 |zs_m - xs_n|^2),
// generated in LDS for each k-tile (64 inducing points m) of the
// workgroup's 64 batch points n; K_uf is never stored.  With the scaling
// c = sqrt(log2(e) / 2), z' = c zs, x' = c xs:
//   K = 2^(log2 sf2 - |z'|^2 - |x'|^2 + (2 z') . x'),
// the dot product on the bf16 matrix cores from hi/lo bf16 splits of 2 z' and
// x' (hi hi + hi lo + lo hi: about 16 significant bits, below the rounding of
// the bf16 / fp16 operand it produces), the accumulator started at
// log2 sf2 - |x'|^2 - |z'|^2 (fp32 norms of the unsplit values), one exp2 per
// entry (the split's rounding can leave a distance of about -1e-5 sf2 relative
// instead of 0, harmless, so there is no clamp).  Inputs per call (written by
// the set-up): Zh, Zl [Mp][KW], zc = -|z'|^2 [Mp], Xh, Xl [Bp][KW],
// xr = log2 sf2 - |x'|^2 [Bp]; KW (16, 32 or 64) >= D, zero
// beyond D; zc and xr are -1e30 on the rows past M and B that a tile covers,
// so those entries are exactly 0 without a mask.  KW = 16 contracts with the 16x16x16 bf16 instruction, else
// 16x16x32 per 32 d.  Each of the 4 waves generates a 32 (m) x 32 (n)
// quadrant: 2 x 2 blocks of 16 x 16, each lane 4 consecutive m of one n,
// stored as one 8-byte LDS write into the swizzled stage layout the fragment
// reads expect.  The z inputs of k-tile j+1 are loaded while tile j is
// generated.
// It carries the side role (SideRows; none with nside = 0).
typedef short s16x4 __attribute__((ext_vector_type(4)));
template <int KW>
struct KufOp {  // one lane's share of a row: 8 bf16, or 4 for KW = 16
  typedef bf16x8 type;
  static constexpr int NC = KW / 32;  // operands per row and lane
  static IFS_DEV f32x4 mma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct KufOp<16> {
  typedef bf16x4 type;
  static constexpr int NC = 1;
  static IFS_DEV f32x4 mma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                      __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
  }
};
template <typename T, int KW>
struct KufGen {
  static constexpr bool kOn = true, kSide = true;
  using Op = typename KufOp<KW>::type;
  static constexpr int NC = KufOp<KW>::NC, RW = 4 * NC;  // operands per row
  const Op *Zh, *Zl;
  const float *zc;
  const Op *Xh, *Xl;
  const float *xr;
  int M, B;
  SideRows rows;
  int side_blocks() const { return rows.nside; }
  IFS_DEV void shift(long o) {
    Zh = gsh(Zh, o); Zl = gsh(Zl, o); zc = gsh(zc, o); Xh = gsh(Xh, o); Xl = gsh(Xl, o);
    xr = gsh(xr, o);
    rows.shift(o);
  }
  IFS_DEV void side(int blk) const { rows.run(blk); }
  template <class C>
  struct State {
    static_assert(C::NW == 4 && C::BN == 64 && C::BK == 64 && C::S == 2,
                  "generator layout: 4 waves, 64 x 64 k-tiles of the B operand, two stages");
    const Op *Zh, *Zl;
    const float *zc;
    int n0, kb, gm, gn, l16, l4;
    Op xh[2][NC], xl[2][NC], zh[2][NC], zl[2][NC];
    f32x4 zcv[2];
    float xrv[2];
    IFS_DEV void init(const KufGen &g, int n0_, int kb_) {
      Zh = g.Zh; Zl = g.Zl; zc = g.zc;
      n0 = n0_;
      kb = kb_;
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      gm = wave >> 1;
      gn = wave & 1;
      l16 = lane & 15;
      l4 = lane >> 4;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const long r = (long)(n0 + gn * 32 + nb * 16 + l16) * RW;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          xh[nb][c] = g.Xh[r + 4 * c + l4];
          xl[nb][c] = g.Xl[r + 4 * c + l4];
        }
        xrv[nb] = g.xr[n0 + gn * 32 + nb * 16 + l16];
      }
    }
    // z inputs of k-tile j
    IFS_DEV void prefetch(int j) {
      const int m0 = kb + j * C::BK + gm * 32;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const long r = (long)(m0 + mb * 16 + l16) * RW;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          zh[mb][c] = Zh[r + 4 * c + l4];
          zl[mb][c] = Zl[r + 4 * c + l4];
        }
        zcv[mb] = *(const f32x4 *)(zc + m0 + mb * 16 + 4 * l4);
      }
    }
    // k-tile j into the stage's B rows (bst = stage + BM rows)
    IFS_DEV void gen(unsigned char *bst, int j) {
      gen_to([&](int ml, int nl, uint2 raw) {
        *(uint2 *)(bst + nl * C::ROWB + (((ml >> 3) ^ (nl & 7)) << 4) + (ml & 7) * 2) = raw;
      });
    }
    // the prefetched k-tile's quadrant: put(ml, nl, raw) receives the entries
    // of inducing points ml .. ml + 3 (tile-local) and batch point nl as four
    // operand-type values
    template <class F>
    IFS_DEV void gen_to(F &&put) {
      wait_vm_lgkm0<0>();
      f32x4 acc[2][2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[mb][nb][q] = zcv[mb][q] + xrv[nb];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            acc[mb][nb] = KufOp<KW>::mma(zh[mb][c], xh[nb][c], acc[mb][nb]);
            acc[mb][nb] = KufOp<KW>::mma(zh[mb][c], xl[nb][c], acc[mb][nb]);
            acc[mb][nb] = KufOp<KW>::mma(zl[mb][c], xh[nb][c], acc[mb][nb]);
          }
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int ml = gm * 32 + mb * 16 + 4 * l4, nl = gn * 32 + nb * 16 + l16;
          T e[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) e[q] = from_f32<T>(__builtin_amdgcn_exp2f(acc[mb][nb][q]));
          uint2 raw;
          __builtin_memcpy(&raw, e, 8);
          put(ml, nl, raw);
        }
    }
  };
};

// The K_uf tiles of KufGen written to memory instead of LDS, in the B operand
// layout of V = L^T K_uf (Kft[n][m], ld >= the padded M), with the same
// arithmetic, so the product over the stored tiles equals the one over the
// generated tiles.  Workgroup t takes k-tile t % nmt (64 inducing points) of
// batch tile t / nmt (64 points).  C: the product's configuration (the
// generator's four-wave quadrant layout).  gs: grouped launch (problem
// blockIdx.z, workspaces gs bytes apart).
template <class C, typename T, int KW>
__global__ __launch_bounds__(C::NT) void k_kuf_gen(KufGen<T, KW> g, T *Kft, long ld, int nmt,
                                                    long gs) {
  if (gs) {
    const long o = goff(gs);
    g.shift(o);
    Kft = gsh(Kft, o);
  }
  const int t = blockIdx.x;
  const int kb = (t % nmt) * 64, n0 = (t / nmt) * 64;
  typename KufGen<T, KW>::template State<C> st;
  st.init(g, n0, kb);
  st.prefetch(0);
  st.gen_to([&](int ml, int nl, uint2 raw) {
    *(uint2 *)(Kft + (long)(n0 + nl) * ld + kb + ml) = raw;
  });
}

// ------------------------------------------------------------------ kernel
template <class C, class EPI, class GEN = NoGen>
__global__ __launch_bounds__(C::NT) void gemm_kernel(Opnd<typename C::T> A,
                                                     Opnd<typename C::T> Bt, Sched sc, EPI epi,
                                                     GEN gen) {
  using T = typename C::T;
  using V = typename Vec16<T>::type;
  constexpr int BM = C::BM, BK = C::BK, S = C::S, ROWB = C::ROWB;
  // loads per wave and stage: A and B rows, or A rows only when B is generated
  constexpr int IPW = GEN::kOn ? BM / (8 * C::NW) : C::IPW;
  static_assert(!GEN::kOn || BM % (8 * C::NW) == 0, "A rows per wave");
  constexpr int TM = C::TM, TN = C::TN;

  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];

  if (sc.gs) {
    const long o = goff(sc.gs);
    A.p = gsh(A.p, o);
    Bt.p = gsh(Bt.p, o);
    sc.skip = gsh(sc.skip, o);
    epi.shift(o);
    gen.shift(o);
  }
  if constexpr (GEN::kSide) {
    const int ntile = sc.sym ? sc.mt * (sc.mt + 1) / 2 : sc.mt * sc.nt;
    if ((int)blockIdx.x >= ntile) {  // uniform across the workgroup
      gen.side((int)blockIdx.x - ntile);
      return;
    }
  }
  int m0, n0, kb, ke, ti;
  sc.tile<C>(blockIdx.x, m0, n0, kb, ke, ti);
  int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (sc.skip && *sc.skip) nk = 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / C::WGN, wn = wave % C::WGN;
  const int lr = lane & 15, kq = lane >> 4;

  // ---- loads: wave w fills combined rows [w*IPW*8, (w+1)*IPW*8) of [A rows; B rows]
  const int drow0 = wave * IPW * 8;
  // lane -> (row lane/8, LDS slot lane%8) holding k-chunk slot ^ row%8
  const int dchunk = (lane & 7) ^ (lane >> 3);
  const T *srcA = A.p + (long)(m0 + (lane >> 3)) * A.ld + dchunk * C::KPL + kb;
  const T *srcB = Bt.p + (long)(n0 - BM + (lane >> 3)) * Bt.ld + dchunk * C::KPL + kb;
  typename GEN::template State<C> gst;
  if constexpr (GEN::kOn) {
    gst.init(gen, n0, kb);
    gst.prefetch(0);
  }
  auto issue = [&](int j) {
    if constexpr (GEN::kOn) gst.gen(smem_raw + (j % S) * C::STAGE + BM * ROWB, j);
    unsigned char *dst = smem_raw + (j % S) * C::STAGE + drow0 * ROWB;
    if constexpr (BM % (8 * IPW) == 0) {
      // every wave's rows lie in one operand: one base pointer and stride
      const bool dA = drow0 < BM;
      const long dld = dA ? A.ld : Bt.ld;
      const T *g = (dA ? srcA : srcB) + (long)drow0 * dld + (long)j * BK;
#pragma unroll
      for (int i = 0; i < IPW; ++i)
        __builtin_amdgcn_global_load_lds((const void *)(g + (long)i * 8 * dld),
                                         (LDS_AS void *)(dst + i * 8 * ROWB), 16, 0, 0);
    } else {
#pragma unroll
      for (int i = 0; i < IPW; ++i) {
        const int R0 = drow0 + 8 * i;
        const T *g = (R0 < BM ? srcA + (long)R0 * A.ld : srcB + (long)R0 * Bt.ld) +
                     (long)j * BK;
        __builtin_amdgcn_global_load_lds((const void *)g, (LDS_AS void *)(dst + i * 8 * ROWB),
                                         16, 0, 0);
      }
    }
    if constexpr (GEN::kOn) {
      if (j + 1 < nk) gst.prefetch(j + 1);
    }
  };

  // ---- fragments: lane reads row lr of a 16-row block, k-chunk 4*sub + kq
  const int sw0 = ((0 + kq) ^ (lr & 7)) * 16, sw1 = ((4 + kq) ^ (lr & 7)) * 16;
  const int aoff = (wm * C::WM + lr) * ROWB, boff = (BM + wn * C::WN + lr) * ROWB;
  V fa[2][2][TM], fb[2][2][TN];  // [register set][k half][tile]
  auto read = [&](auto set_c, int j) {
    constexpr int SET = decltype(set_c)::value;
    const unsigned char *st = smem_raw + (j % S) * C::STAGE;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int sw = h ? sw1 : sw0;
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[SET][h][i] = *(const V *)(st + aoff + i * 16 * ROWB + sw);
#pragma unroll
      for (int j2 = 0; j2 < TN; ++j2) fb[SET][h][j2] = *(const V *)(st + boff + j2 * 16 * ROWB + sw);
    }
  };

  typename C::Acc acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = typename C::Acc{0, 0, 0, 0};
  auto mma = [&](auto set_c, int h) {
    constexpr int SET = decltype(set_c)::value;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = mfma16(fa[SET][h][i], fb[SET][h][j], acc[i][j]);
  };
  // one k-tile: first half of its MFMAs, then (if there is a next k-tile) wait
  // for it, refill the stage this k-tile vacated, read the next fragments, and
  // issue the second half while those reads are in flight
  auto step = [&](auto cur_c, int it) {
    constexpr int CUR = decltype(cur_c)::value;
    mma(cur_c, 0);
    if (it + 1 < nk) {
      __builtin_amdgcn_sched_barrier(0);
      wait_stages<IPW, S - 2>(min(nk - it - 2, S - 2));
      __builtin_amdgcn_s_barrier();
      if (it + S < nk) issue(it + S);
      read(IC<1 - CUR>{}, it + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
    mma(cur_c, 1);
  };

  if (nk > 0) {
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (j < nk) issue(j);
    wait_stages<IPW, S - 1>(min(nk, S) - 1);
    __builtin_amdgcn_s_barrier();
    read(IC<0>{}, 0);
    int it = 0;
    for (; it + 1 < nk; it += 2) {
      step(IC<0>{}, it);
      step(IC<1>{}, it + 1);
    }
    if (it < nk) step(IC<0>{}, it);
  }
  __syncthreads();
  TileInfo t{m0, n0, ti, (int)blockIdx.y};
  if constexpr (EpiTakesRegs<EPI>::value) {
    epi.template run_regs<C>(acc, (float *)smem_raw, t);
  } else {
    // stage the fp32 accumulator tile in LDS: Cs[r][c], r < BM, c < BN
    float *Cs = (float *)smem_raw;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Cs[(wm * C::WM + i * 16 + (C::A64 ? 4 * q + kq : 4 * kq + q)) * C::LDC + wn * C::WN +
             j * 16 + lr] = (float)acc[i][j][q];
    __syncthreads();
    epi.template run<C>(Cs, t);
  }
}

// Where and how to launch: the stream, and optionally two events that the
// dispatch itself stamps at kernel start and end (per-kernel timing without
// the cost of separately recorded events).
struct Launch {
  hipStream_t st;
  hipEvent_t t0, t1;
  int groups;  // problems of a grouped launch (0 or 1: one problem)
  long gs;     // bytes between their workspaces
};

// Host-side launch helper.  extra: LDS bytes the epilogue needs beyond the
// staged tile and its scratch.
template <class C, class EPI, class GEN = NoGen>
static inline hipError_t launch_gemm(const Launch &lc, const Opnd<typename C::T> &A,
                                     const Opnd<typename C::T> &Bt, const Sched &sc,
                                     const EPI &epi, int extra = 0, const GEN &gen = GEN{}) {
  const int ntile = sc.sym ? sc.mt * (sc.mt + 1) / 2 : sc.mt * sc.nt;
  if (ntile <= 0) return hipSuccess;
  dim3 grid(ntile + gen.side_blocks(), sc.nsplit > 1 ? sc.nsplit : 1,
            lc.groups > 1 ? lc.groups : 1);
  auto kern = gemm_kernel<C, EPI, GEN>;
  Sched sg = sc;
  sg.gs = lc.groups > 1 ? lc.gs : 0;
  const int smem = C::smem(extra);
  static int attr_bytes = 0;
  if (smem > attr_bytes) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, smem);
    if (e != hipSuccess) return e;
    attr_bytes = smem;
  }
  if (lc.t0)
    hipExtLaunchKernelGGL(kern, grid, dim3(C::NT), smem, lc.st, lc.t0, lc.t1, 0, A, Bt, sg, epi,
                          gen);
  else
    hipLaunchKernelGGL(kern, grid, dim3(C::NT), smem, lc.st, A, Bt, sg, epi, gen);
  return hipGetLastError();
}
