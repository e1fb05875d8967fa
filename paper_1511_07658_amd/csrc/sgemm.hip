// SGEMM C = A B (Table 3 "MM", single precision) for the GVM on gfx950:
// FP32 MFMA (v_mfma_f32_32x32x2_f32) on LDS-staged, double-buffered tiles,
// as one grouped persistent launch over the tiles of every request of the
// group.  The unit -> request map is a search over the per-request first tile
// held in the kernel arguments; a tile is always computed by the same code in
// the same order, whatever else is in the group, so a rank's C is
// bit-identical alone and in the mix.
#include "gemm_balance.hpp"
#include "group_device.hpp"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

namespace gvm {

namespace {

// ---------------------------------------------------------------- SGEMM
//
// Workgroup tile BM x BN, k-step BK, WM x WN waves; each wave owns a
// (BM/WM) x (BN/WN) block of C as (BM/WM/32) x (BN/WN/32) accumulators of
// one 32x32 MFMA each.  v_mfma_f32_32x32x2_f32 multiplies a 32x2 slice of A
// by a 2x32 slice of B; lane l supplies A[l%32][k(l)] and B[k(l)][l%32] and
// lane group g = l/32 selects which of the two k values it carries.  Each
// run of eight k (8m .. 8m + 7) feeds four MFMA steps, with the k pairs
// (8m + t, 8m + 4 + t) for t = 0 .. 3, g = 0 the smaller k: every C element
// sums the pairs (0, 4), (1, 5), (2, 6), (3, 7), (8, 12), ... in that order
// into one accumulator whatever the tile configuration, so all
// configurations give the same bits and requests of any sizes may share one
// launch.
//
// In LDS the k index of a tile is stored permuted, so that the KH = BK/2
// values a lane multiplies in the KH steps of a tile sit side by side: k =
// 8m + 4h + t (h in {0, 1}, t in 0 .. 3) goes to k' = h * KH + 4m + t.  A
// run of four k stays contiguous, so a fetched float4 is still one 16-byte
// LDS write, to the same banks as without the permutation.  A sits as
// As[m][k'] (rows padded by 4 floats), and a lane's A fragments of a whole
// tile are read with 16-byte LDS reads.  B has two stagings, chosen per tile
// configuration by the tuner:
//  * BT: Bs[n][k'], B transposed on the way in (each thread fetches four
//    k-rows of one column, coalesced along n); B fragments are then 16-byte
//    reads like A's;
//  * row-major: Bs[k'][n] from float4 loads along n (k-row k goes to row
//    k'); B fragments are 4-byte reads (one per MFMA step and column block),
//    the two lane groups on rows BK/2 apart.
// All fragments of a k-step are read before its MFMAs.  Double buffering:
// the next tile is fetched into registers at the start of a k-step and
// written to the other LDS buffer half-way through the MFMAs, so one barrier
// per k-step remains.  Interior tiles take unchecked loads and stores; edge
// tiles check every element and read zeros outside the matrix.
//
// PIPE variant: the fragments of the next k-tile are read from LDS into a
// second register set while the MFMAs of the current one run, so no k-step
// starts by waiting for LDS.  Tile t is written to LDS buffer t % 2 during
// step t - 2, its fragments read during step t - 1 and multiplied in step t;
// one barrier at the end of each step orders both hazards (a write of tile
// t + 2 follows every read of tile t, which shares its buffer; a read of
// tile t + 1 follows every write of it).  Tile 0's fragments are read in the
// prologue, so a barrier follows them before step 0 writes tile 2.  The k
// order of every C element is the same as without PIPE.
//
// Persistent grid, XCD-aware: the units (tiles, requests in order, tiles of a
// request row-major) are dealt to the 8 XCDs in contiguous blocks, so that
// tiles sharing rows of A and columns of B share an L2.
//
// Balanced grid (mixed sizes, one workgroup per tile): the blocks are cut by
// work instead of by count.  The requests come largest first, so equal
// counts would give the first XCD the longest tiles and the last one the
// shortest.  The units are cut into 16 contiguous slices of equal k-step
// work instead, and XCD x takes slice x from the long end and then slice
// 15 - x from the short end, so every XCD ends on short tiles; the grid
// holds as many workgroups per XCD as the longest pair has units (the rest
// exit at once).

// MINW: the waves per SIMD the register allocation must leave room for (1:
// no constraint); the compiler then keeps VGPRs + AGPRs within 512 / MINW.
template <int BM, int BN, int BK, int WM, int WN, bool BT, int DEPTH, bool VEC, bool PIPE, int MINW>
__global__ __launch_bounds__(WM * WN * 64) __attribute__((amdgpu_waves_per_eu(MINW))) void sgemm_group_kernel(
    GemmGroup g) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 32, FN = TN / 32;
  constexpr int KH = BK / 2;
  constexpr int AST = BK + 4;                      // LDS row stride of As
  constexpr int BST = BT ? BK + 4 : BN + 4;        // LDS row stride of Bs
  constexpr int A4 = BM * BK / 4 / NT;             // float4 of A per thread per tile
  constexpr int B4 = BK * BN / 4 / NT;             // float4 of B per thread per tile
  static_assert(TM % 32 == 0 && TN % 32 == 0, "wave tile must be a multiple of 32");
  static_assert(KH % 4 == 0, "BK must be a multiple of 8");
  static_assert(A4 >= 1 && B4 >= 1 && A4 * NT * 4 == BM * BK && B4 * NT * 4 == BK * BN, "tile/threads mismatch");
  static_assert(DEPTH >= 1 && DEPTH <= 3, "global prefetch depth is one to three k-tiles");
  static_assert(!PIPE || DEPTH <= 2, "the pipelined loop takes a fetch depth of one or two");

  __shared__ __attribute__((aligned(16))) float As[2][BM * AST];
  __shared__ __attribute__((aligned(16))) float Bs[2][BT ? BN * BST : BK * BST];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int li = lane & 31, lg = lane >> 5;

  // XCD-aware order: with G a multiple of 8, workgroup w runs on XCD w % 8;
  // renumbering it v = (w % 8) * (G / 8) + w / 8 gives each XCD a contiguous
  // block of units in every round of the stride loop below.
  const uint32_t G = gridDim.x;
  const uint32_t U = g.total_units;
  uint32_t v = blockIdx.x;
  if (G % kXcds == 0) v = (blockIdx.x % kXcds) * (G / kXcds) + blockIdx.x / kXcds;

  uint32_t u0 = v, uend = U, ustep = G;
  if (g.balanced) {
    // the j-th workgroup of XCD x takes the j-th unit of the XCD's two
    // slices; the grid holds as many per XCD as the longest pair has units
    // (the slices of xcd_slices(): 2x and 2x + 1, or x and 15 - x when paired)
    const int x = static_cast<int>(blockIdx.x % kXcds);
    const int s0 = g.balanced == 2 ? x : 2 * x;
    const int s1 = g.balanced == 2 ? kGemmSlices - 1 - x : 2 * x + 1;
    const uint32_t j = blockIdx.x / kXcds;
    const uint32_t len0 = g.cut[s0 + 1] - g.cut[s0];
    u0 = j < len0 ? g.cut[s0] + j : g.cut[s1] + (j - len0);
    uend = j < len0 ? g.cut[s0 + 1] : g.cut[s1 + 1];
    ustep = uend;  // one unit per workgroup
  }
  for (uint32_t u = u0; u < uend; u += ustep) {
    const int q = find_request(g, u);
    const GemmDesc& d = g.d[q];
    const int n = static_cast<int>(d.n);
    const uint32_t local = u - d.unit_begin;
    const int row0 = static_cast<int>(local / d.tiles_n) * BM;
    const int col0 = static_cast<int>(local % d.tiles_n) * BN;
    const float* __restrict__ A = d.A;
    const float* __restrict__ B = d.B;
    const bool rows_in = row0 + BM <= n, cols_in = col0 + BN <= n;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{0};

    // 4 consecutive floats of row r from column c, or zeros outside n x n
    auto row4 = [&](const float* M, int r, int c, bool fast) -> f32x4 {
      const float* p = M + static_cast<size_t>(r) * n + c;
      if (fast) {
        if (VEC) return *reinterpret_cast<const f32x4*>(p);
        return f32x4{p[0], p[1], p[2], p[3]};
      }
      f32x4 x = f32x4{0};
      if (VEC) {
        // n and c are multiples of 4: a group of four lies wholly inside or
        // wholly outside the matrix, so one check and one 16-byte load
        if (r < n && c < n) x = *reinterpret_cast<const f32x4*>(p);
        return x;
      }
      if (r < n) {
        if (c + 0 < n) x.x = p[0];
        if (c + 1 < n) x.y = p[1];
        if (c + 2 < n) x.z = p[2];
        if (c + 3 < n) x.w = p[3];
      }
      return x;
    };

    // DEPTH register slots of fetched k-tiles (slot index is a compile-time tag)
    f32x4 ra[DEPTH][A4], rb[DEPTH][B4];
    // FAST (a compile-time tag): an interior tile, every load unchecked
    auto load_tile = [&](int k0, auto slot_tag, auto fast_tag) {
      constexpr int SL = decltype(slot_tag)::value;
      constexpr bool FAST = decltype(fast_tag)::value;
      const bool k_in = FAST || k0 + BK <= n;
#pragma unroll
      for (int i = 0; i < A4; ++i) {
        const int f = tid + i * NT;
        ra[SL][i] = row4(A, row0 + f / (BK / 4), k0 + (f % (BK / 4)) * 4, FAST || (rows_in && k_in));
      }
      if (BT) {
#pragma unroll
        for (int i = 0; i < B4; ++i) {  // four k-rows of one column
          const int f = tid + i * NT;
          const int c = f % BN, kq = f / BN;
          const int gr = k0 + 4 * kq, gc = col0 + c;
          const float* p = B + static_cast<size_t>(gr) * n + gc;
          if (FAST || (cols_in && k_in)) {
            rb[SL][i] = f32x4{p[0], p[n], p[2 * n], p[3 * n]};
          } else if (VEC) {
            // n and gr are multiples of 4: the four k-rows are all in or all out
            rb[SL][i] = (gc < n && gr < n) ? f32x4{p[0], p[n], p[2 * n], p[3 * n]} : f32x4{0};
          } else {
            f32x4 x = f32x4{0};
            if (gc < n) {
              if (gr + 0 < n) x.x = p[0];
              if (gr + 1 < n) x.y = p[n];
              if (gr + 2 < n) x.z = p[2 * static_cast<size_t>(n)];
              if (gr + 3 < n) x.w = p[3 * static_cast<size_t>(n)];
            }
            rb[SL][i] = x;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < B4; ++i) {  // four columns of one k-row
          const int f = tid + i * NT;
          rb[SL][i] = row4(B, k0 + f / (BN / 4), col0 + (f % (BN / 4)) * 4, FAST || (cols_in && k_in));
        }
      }
    };
    // k-permuted LDS layout: the float4 of k = 4q .. 4q + 3 goes to k' =
    // (q % 2) * KH + 4 (q / 2) .. + 3
    auto store_tile = [&](int buf, auto slot_tag) {
      constexpr int SL = decltype(slot_tag)::value;
#pragma unroll
      for (int i = 0; i < A4; ++i) {
        const int f = tid + i * NT;
        const int r = f / (BK / 4), q = f % (BK / 4);
        *reinterpret_cast<f32x4*>(&As[buf][r * AST + (q & 1) * KH + 4 * (q >> 1)]) = ra[SL][i];
      }
#pragma unroll
      for (int i = 0; i < B4; ++i) {
        const int f = tid + i * NT;
        if (BT) {
          const int c = f % BN, kq = f / BN;
          *reinterpret_cast<f32x4*>(&Bs[buf][c * BST + (kq & 1) * KH + 4 * (kq >> 1)]) = rb[SL][i];
        } else {
          const int r = f / (BN / 4), c = (f % (BN / 4)) * 4;
          const int rp = ((r >> 2) & 1) * KH + ((r >> 3) << 2) + (r & 3);
          *reinterpret_cast<f32x4*>(&Bs[buf][rp * BST + c]) = rb[SL][i];
        }
      }
    };

    const int ktiles = (n + BK - 1) / BK;
    // One k-step: MFMAs on LDS buffer kt & 1.  Tile kt + 1 (in register
    // slot `cur`) is written to the other buffer half-way through.  With
    // DEPTH 1 its fetch is issued at the start of the same step, so a fetch
    // has half a k-step to arrive; with DEPTH > 1 the step first issues the
    // fetch of tile kt + DEPTH into slot `nxt` (tile kt's, written to LDS
    // in the previous step), so a fetch has DEPTH - 1/2 k-steps.  Tile t
    // lives in slot t % DEPTH.
    //
    // On an interior tile whose k-tiles divide evenly (FAST), every step
    // issues the same loads and LDS writes without a branch: the last steps
    // fetch the last k-tile again and write it to the buffer no later step
    // reads.  The compiler can then wait for exactly the fetch it needs
    // (`s_waitcnt vmcnt(n)` with the newer fetch still in flight); with
    // conditional fetches it waits for all of them (`vmcnt(0)`), which
    // takes the fetch depth back to half a k-step.
    auto step = [&](int kt, auto cur, auto nxt, auto fast_tag) {
      constexpr bool FAST = decltype(fast_tag)::value;
      const int buf = kt & 1;
      const bool more = FAST || kt + 1 < ktiles;
      if constexpr (FAST) {
        const int kf = min(kt + DEPTH, ktiles - 1) * BK;
        if constexpr (DEPTH == 1) load_tile(kf, cur, fast_tag);
        else load_tile(kf, nxt, fast_tag);
      } else if (DEPTH == 1) {
        if (more) load_tile((kt + 1) * BK, cur, fast_tag);
      } else if (kt + DEPTH < ktiles) {
        load_tile((kt + DEPTH) * BK, nxt, fast_tag);
      }
      float af[FM][KH], bf[FN][KH];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const float* src = &As[buf][(wm * TM + i * 32 + li) * AST + lg * KH];
#pragma unroll
        for (int j = 0; j < KH; j += 4) {
          const f32x4 x = *reinterpret_cast<const f32x4*>(src + j);
          af[i][j] = x.x; af[i][j + 1] = x.y; af[i][j + 2] = x.z; af[i][j + 3] = x.w;
        }
      }
#pragma unroll
      for (int i = 0; i < FN; ++i) {
        if (BT) {
          const float* src = &Bs[buf][(wn * TN + i * 32 + li) * BST + lg * KH];
#pragma unroll
          for (int j = 0; j < KH; j += 4) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(src + j);
            bf[i][j] = x.x; bf[i][j + 1] = x.y; bf[i][j + 2] = x.z; bf[i][j + 3] = x.w;
          }
        } else {
          const float* src = &Bs[buf][(lg * KH) * BST + wn * TN + i * 32 + li];
#pragma unroll
          for (int j = 0; j < KH; ++j) bf[i][j] = src[j * BST];
        }
      }
#pragma unroll
      for (int s = 0; s < KH; ++s) {
        // The other buffer was last read before the previous barrier.
        if (s == KH / 2 && more) store_tile(buf ^ 1, cur);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    };

    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1 % DEPTH>;
    using S2 = std::integral_constant<int, 2 % DEPTH>;
    auto run = [&](auto fast_tag) {
      constexpr bool FAST = decltype(fast_tag)::value;
      load_tile(0, S0{}, fast_tag);
      store_tile(0, S0{});
      if constexpr (DEPTH >= 2) {
        if (FAST || ktiles > 1) load_tile(min(1, ktiles - 1) * BK, S1{}, fast_tag);
      }
      if constexpr (DEPTH >= 3) {
        if (FAST || ktiles > 2) load_tile(min(2, ktiles - 1) * BK, S2{}, fast_tag);
      }
      __syncthreads();
      // DEPTH steps per trip, so that every slot index is a compile-time tag
      for (int kt = 0; kt < ktiles; kt += DEPTH) {
        step(kt, S1{}, S0{}, fast_tag);
        if constexpr (DEPTH >= 2) {
          if (FAST || kt + 1 < ktiles) step(kt + 1, S2{}, S1{}, fast_tag);
        }
        if constexpr (DEPTH >= 3) {
          if (FAST || kt + 2 < ktiles) step(kt + 2, S0{}, S2{}, fast_tag);
        }
      }
    };
    // ---- PIPE: fragments of tile kt + 1 read during the MFMAs of tile kt
    float pa[2][FM][KH], pb[2][FN][KH];
    auto read_frags = [&](int buf, auto fset_tag) {
      constexpr int F = decltype(fset_tag)::value;
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const float* src = &As[buf][(wm * TM + i * 32 + li) * AST + lg * KH];
#pragma unroll
        for (int j = 0; j < KH; j += 4) {
          const f32x4 x = *reinterpret_cast<const f32x4*>(src + j);
          pa[F][i][j] = x.x; pa[F][i][j + 1] = x.y; pa[F][i][j + 2] = x.z; pa[F][i][j + 3] = x.w;
        }
      }
#pragma unroll
      for (int i = 0; i < FN; ++i) {
        if (BT) {
          const float* src = &Bs[buf][(wn * TN + i * 32 + li) * BST + lg * KH];
#pragma unroll
          for (int j = 0; j < KH; j += 4) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(src + j);
            pb[F][i][j] = x.x; pb[F][i][j + 1] = x.y; pb[F][i][j + 2] = x.z; pb[F][i][j + 3] = x.w;
          }
        } else {
          const float* src = &Bs[buf][(lg * KH) * BST + wn * TN + i * 32 + li];
#pragma unroll
          for (int j = 0; j < KH; ++j) pb[F][i][j] = src[j * BST];
        }
      }
    };
    // Step kt: MFMAs of tile kt (fragment set `fc`), fragments of tile
    // kt + 1 into set `fn`; half-way, tile kt + 2 (register slot `ws`) goes
    // to LDS buffer kt % 2 and the fetch of tile kt + 2 + DEPTH takes its
    // slot.  FAST: the same instructions every step, indexes clamped to the
    // last k-tile (the extra reads and writes land where no step uses them).
    //
    // The MFMAs touch no memory, so the compiler may move them across the
    // barrier; the two empty asm statements keep each step's MFMAs between
    // the LDS reads of the next fragments and the step's barrier (the first
    // makes the current fragments appear to change after the reads, the
    // second makes the last MFMA of each accumulator chain appear to be read
    // before the barrier), so the barrier's wait for those reads is covered
    // by the step's MFMAs.
    auto step_pipe = [&](int kt, auto fc, auto fn, auto ws, auto fast_tag) {
      constexpr bool FAST = decltype(fast_tag)::value;
      constexpr int FC = decltype(fc)::value;
      const int buf = kt & 1;
      if (FAST || kt + 1 < ktiles) read_frags(buf ^ 1, fn);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int s = 0; s < KH; ++s) asm volatile("" : "+v"(pa[FC][i][s])::"memory");
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int s = 0; s < KH; ++s) asm volatile("" : "+v"(pb[FC][j][s])::"memory");
#pragma unroll
      for (int s = 0; s < KH; ++s) {
        if (s == KH / 2 && (FAST || kt + 2 < ktiles)) {
          store_tile(buf, ws);
          if constexpr (FAST) load_tile(min(kt + 2 + DEPTH, ktiles - 1) * BK, ws, fast_tag);
          else if (kt + 2 + DEPTH < ktiles) load_tile((kt + 2 + DEPTH) * BK, ws, fast_tag);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[FC][i][s], pb[FC][j][s], acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) asm volatile("" ::"v"(acc[i][j][15]) : "memory");
      __syncthreads();
    };
    using F0 = std::integral_constant<int, 0>;
    using F1 = std::integral_constant<int, 1>;
    using W0 = std::integral_constant<int, 2 % DEPTH>;   // slot of tile kt + 2, kt even
    using W1 = std::integral_constant<int, 3 % DEPTH>;   // slot of tile kt + 3
    auto run_pipe = [&](auto fast_tag) {
      constexpr bool FAST = decltype(fast_tag)::value;
      load_tile(0, S0{}, fast_tag);
      store_tile(0, S0{});
      if (FAST || ktiles > 1) {
        load_tile(min(1, ktiles - 1) * BK, S1{}, fast_tag);
        store_tile(1, S1{});
      }
      // tiles 2 .. 1 + DEPTH into their slots
      if (FAST || ktiles > 2) load_tile(min(2, ktiles - 1) * BK, W0{}, fast_tag);
      if constexpr (DEPTH >= 2) {
        if (FAST || ktiles > 3) load_tile(min(3, ktiles - 1) * BK, W1{}, fast_tag);
      }
      __syncthreads();
      read_frags(0, F0{});
      // step 0 writes tile 2 over tile 0's buffer: every wave must have read
      // tile 0's fragments first
      __syncthreads();
      for (int kt = 0; kt < ktiles; kt += 2) {
        step_pipe(kt, F0{}, F1{}, W0{}, fast_tag);
        if (FAST || kt + 1 < ktiles) step_pipe(kt + 1, F1{}, F0{}, W1{}, fast_tag);
      }
    };
    if constexpr (PIPE) {
      if (rows_in && cols_in && n % BK == 0 && ktiles % 2 == 0) run_pipe(std::true_type{});
      else run_pipe(std::false_type{});
    } else {
      if (rows_in && cols_in && n % BK == 0 && ktiles % DEPTH == 0) run(std::true_type{});
      else run(std::false_type{});
    }

    float* __restrict__ C = d.C;
    if (rows_in && cols_in) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = col0 + wn * TN + j * 32 + li;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = row0 + wm * TM + i * 32 + 8 * (r / 4) + 4 * lg + (r % 4);
            C[static_cast<size_t>(row) * n + col] = acc[i][j][r];
          }
        }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int col = col0 + wn * TN + j * 32 + li;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = row0 + wm * TM + i * 32 + 8 * (r / 4) + 4 * lg + (r % 4);
            if (row < n && col < n) C[static_cast<size_t>(row) * n + col] = acc[i][j][r];
          }
        }
    }
  }
}

// Tile configurations.  Index order is part of the tuner table format.
const GemmConfig kGemmConfigs[] = {
    {0, 64, 64, 16, 2, 2, true},
    {1, 128, 64, 16, 2, 2, true},
    {2, 128, 128, 16, 2, 2, true},
    {3, 128, 128, 32, 2, 2, true},
    {4, 256, 128, 16, 4, 2, true},
    {5, 128, 256, 16, 2, 4, true},
    {6, 256, 128, 32, 4, 2, true},
    {7, 64, 128, 16, 2, 2, true},
    {8, 128, 128, 16, 2, 2, false},
    {9, 256, 128, 16, 4, 2, false},
    {10, 128, 256, 16, 2, 4, false},
    {11, 256, 128, 32, 4, 2, false},
    {12, 128, 128, 32, 2, 2, false},
    {13, 64, 128, 16, 2, 2, false},
    // row-major B tiles with two k-tiles fetched ahead (prefetch depth 2)
    {14, 256, 128, 16, 4, 2, false},
    {15, 128, 128, 16, 2, 2, false},
    {16, 256, 128, 32, 4, 2, false},
    {17, 64, 128, 16, 2, 2, false},
    {18, 128, 128, 32, 2, 2, false},
    // three k-tiles fetched ahead
    {19, 256, 128, 16, 4, 2, false},
    {20, 256, 128, 32, 4, 2, false},
    {21, 128, 128, 16, 2, 2, false},
    // fragments of the next k-tile read during the current MFMAs (PIPE), two ahead
    {22, 256, 128, 16, 4, 2, false},
    {23, 128, 128, 32, 2, 2, false},
    {24, 128, 128, 16, 2, 2, false},
    {25, 64, 128, 16, 2, 2, false},
    // the same with one k-tile fetched ahead (a fetch still has a whole step)
    {26, 256, 128, 16, 4, 2, false},
    // larger tiles for large n, two ahead
    {27, 128, 256, 32, 2, 4, false},
    {28, 256, 256, 16, 4, 2, false},
    // two ahead with registers held to four waves per SIMD (VGPRs + AGPRs <= 128)
    {29, 64, 128, 16, 2, 2, false},
};
constexpr int kNumGemmConfigs = sizeof(kGemmConfigs) / sizeof(kGemmConfigs[0]);

int g_forced_config = -1;

#include "gemm_tiles.inc"   // kTileTable: (n_max, config index) rows written by the tuner

template <int BM, int BN, int BK, int WM, int WN, bool BT, int DEPTH = 1, bool PIPE = false, int MINW = 1>
hipError_t launch_cfg(const GemmGroup& g, bool vec, hipStream_t s, int grid_cap) {
  constexpr int NT = WM * WN * 64;
  int cap = grid_cap > 0 ? grid_cap : 256 * 2;
  int grid = static_cast<int>(std::min<uint32_t>(g.total_units, static_cast<uint32_t>(cap)));
  if (grid > kXcds) grid -= grid % kXcds;  // whole rounds over the 8 XCDs
  if (g.balanced) {  // one workgroup per unit of the longest XCD pair of slices
    uint32_t most = 0;
    for (int x = 0; x < kXcds; ++x) {
      int s0, s1;
      xcd_slices(x, g.balanced == 2, &s0, &s1);
      most = std::max(most, (g.cut[s0 + 1] - g.cut[s0]) + (g.cut[s1 + 1] - g.cut[s1]));
    }
    grid = static_cast<int>(most) * kXcds;
  }
  return vec ? launch_group(sgemm_group_kernel<BM, BN, BK, WM, WN, BT, DEPTH, true, PIPE, MINW>, grid, NT, s, g)
             : launch_group(sgemm_group_kernel<BM, BN, BK, WM, WN, BT, DEPTH, false, PIPE, MINW>, grid, NT, s, g);
}

}  // namespace

int gemm_config_count() { return kNumGemmConfigs; }
const GemmConfig& gemm_config(int idx) { return kGemmConfigs[idx]; }
void gemm_config_force(int idx) { g_forced_config = (idx >= 0 && idx < kNumGemmConfigs) ? idx : -1; }

int gemm_config_for(uint64_t n) {
  if (g_forced_config >= 0) return g_forced_config;
  // tuning and tests only: force one configuration for every size
  if (const char* env = getenv("GVM_SGEMM_CONFIG")) {
    const int c = atoi(env);
    if (c >= 0 && c < kNumGemmConfigs) return c;
  }
  int c = static_cast<int>(kTileTable[sizeof(kTileTable) / sizeof(kTileTable[0]) - 1][1]);
  for (const auto& row : kTileTable)
    if (n <= row[0]) {
      c = static_cast<int>(row[1]);
      break;
    }
  return c;
}
void finalize_gemm_group(GemmGroup& g, int config_idx) {
  const GemmConfig& c = kGemmConfigs[config_idx];
  uint32_t u = 0;
  for (uint32_t i = 0; i < g.count; ++i) {
    const uint32_t n = g.d[i].n;
    const uint32_t tm = (n + c.bm - 1) / c.bm, tn = (n + c.bn - 1) / c.bn;
    g.d[i].tiles_n = tn;
    g.d[i].unit_begin = u;
    g.d[i].units = tm * tn;
    u += tm * tn;
  }
  g.total_units = u;
  uint32_t units[kMaxGroup], ksteps[kMaxGroup];
  for (uint32_t i = 0; i < g.count; ++i) {
    units[i] = g.d[i].units;
    ksteps[i] = (g.d[i].n + c.bk - 1) / c.bk;
  }
  balance_slices(g.count, units, ksteps, g.cut);
  g.balanced = 0;
}
hipError_t launch_sgemm_group(const GemmGroup& g_in, int config_idx, hipStream_t s, int grid_cap) {
  GemmGroup g = g_in;
  g.balanced = 0;
  if (grid_cap > 0 && static_cast<uint32_t>(grid_cap) >= g.total_units && g.count > 1) {
    bool mixed = false;
    for (uint32_t i = 1; i < g.count; ++i) mixed |= g.d[i].n != g.d[0].n;
    // GVM_SGEMM_XCD_PAIRED=0 keeps each XCD on one contiguous run (tuning)
    static const bool paired = [] {
      const char* e = getenv("GVM_SGEMM_XCD_PAIRED");
      return !(e && e[0] == '0');
    }();
    if (mixed) g.balanced = paired ? 2 : 1;
  }
  bool vec = true;
  for (uint32_t i = 0; i < g.count; ++i)
    if ((g.d[i].n % 4) != 0 || (reinterpret_cast<uintptr_t>(g.d[i].A) & 15) ||
        (reinterpret_cast<uintptr_t>(g.d[i].B) & 15))
      vec = false;
  switch (config_idx) {
    case 0: return launch_cfg<64, 64, 16, 2, 2, true>(g, vec, s, grid_cap);
    case 1: return launch_cfg<128, 64, 16, 2, 2, true>(g, vec, s, grid_cap);
    case 2: return launch_cfg<128, 128, 16, 2, 2, true>(g, vec, s, grid_cap);
    case 3: return launch_cfg<128, 128, 32, 2, 2, true>(g, vec, s, grid_cap);
    case 4: return launch_cfg<256, 128, 16, 4, 2, true>(g, vec, s, grid_cap);
    case 5: return launch_cfg<128, 256, 16, 2, 4, true>(g, vec, s, grid_cap);
    case 6: return launch_cfg<256, 128, 32, 4, 2, true>(g, vec, s, grid_cap);
    case 7: return launch_cfg<64, 128, 16, 2, 2, true>(g, vec, s, grid_cap);
    case 8: return launch_cfg<128, 128, 16, 2, 2, false>(g, vec, s, grid_cap);
    case 9: return launch_cfg<256, 128, 16, 4, 2, false>(g, vec, s, grid_cap);
    case 10: return launch_cfg<128, 256, 16, 2, 4, false>(g, vec, s, grid_cap);
    case 11: return launch_cfg<256, 128, 32, 4, 2, false>(g, vec, s, grid_cap);
    case 12: return launch_cfg<128, 128, 32, 2, 2, false>(g, vec, s, grid_cap);
    case 13: return launch_cfg<64, 128, 16, 2, 2, false>(g, vec, s, grid_cap);
    case 14: return launch_cfg<256, 128, 16, 4, 2, false, 2>(g, vec, s, grid_cap);
    case 15: return launch_cfg<128, 128, 16, 2, 2, false, 2>(g, vec, s, grid_cap);
    case 16: return launch_cfg<256, 128, 32, 4, 2, false, 2>(g, vec, s, grid_cap);
    case 17: return launch_cfg<64, 128, 16, 2, 2, false, 2>(g, vec, s, grid_cap);
    case 18: return launch_cfg<128, 128, 32, 2, 2, false, 2>(g, vec, s, grid_cap);
    case 19: return launch_cfg<256, 128, 16, 4, 2, false, 3>(g, vec, s, grid_cap);
    case 20: return launch_cfg<256, 128, 32, 4, 2, false, 3>(g, vec, s, grid_cap);
    case 21: return launch_cfg<128, 128, 16, 2, 2, false, 3>(g, vec, s, grid_cap);
    case 22: return launch_cfg<256, 128, 16, 4, 2, false, 2, true>(g, vec, s, grid_cap);
    case 23: return launch_cfg<128, 128, 32, 2, 2, false, 2, true>(g, vec, s, grid_cap);
    case 24: return launch_cfg<128, 128, 16, 2, 2, false, 2, true>(g, vec, s, grid_cap);
    case 25: return launch_cfg<64, 128, 16, 2, 2, false, 2, true>(g, vec, s, grid_cap);
    case 26: return launch_cfg<256, 128, 16, 4, 2, false, 1, true>(g, vec, s, grid_cap);
    case 27: return launch_cfg<128, 256, 32, 2, 4, false, 2>(g, vec, s, grid_cap);
    case 28: return launch_cfg<256, 256, 16, 4, 2, false, 2>(g, vec, s, grid_cap);
    case 29: return launch_cfg<64, 128, 16, 2, 2, false, 2, false, 4>(g, vec, s, grid_cap);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gvm
