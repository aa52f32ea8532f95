// Lattice random-walk replication engines (paper section 5.1, third model).
//
// WAVE mapping: one replication per wavefront, lane w = walker w. The
// replication's visited-site bitmap (grid^2 bits, 512 B at 64x64) lives in
// LDS and every move sets its bit with an LDS atomic or; at the end the
// lanes popcount the bitmap and sum squared displacements across the wave.
//
// With few replications that form leaves the chip idle and each wave walks
// its 1000 steps one after the other. The walk is a prefix sum of
// independent moves, so rw_seg_kernel cuts every walker's steps into 16
// segments, one lane each (a workgroup per replication): pass 1 counts a
// segment's net displacement (popcounts of the move fields), a 16-lane
// exclusive scan gives each segment its start, and pass 2 replays the
// segment from there, marking the sites. Both forms give identical outputs;
// the launcher picks by the number of replications.
//
// Optionally (PW) every walker also marks a bitmap of its own, in global
// memory, and output 2 is the sum over walkers of their popcounts.
//
// SIMT mapping: one replication per lane; the lane walks its walkers one
// after the other and keeps the replication's bitmap in global memory, the
// per-thread state the paper's thread-per-replication form implies. The
// same kernel with one working lane per wavefront is the paper's own WLP.
//
// On taus88 streams (RNG = RNG_TAUS88) move t of walker w takes bits
// 2(t&15) of output w ceil(T/16) + (t>>4) of the replication's stream: each
// walker reads a contiguous run, so a WAVE lane jumps to its walker's run and
// a SIMT lane reads the stream in order, walker after walker.
#include "device.hpp"
#include "kernels.hpp"
#include "taus.hpp"

namespace mrip {

namespace {

// Move d (0:+x 1:-x 2:+y 3:-y) as two sign-extended 2-bit fields of small
// tables: dx = field d of 0b00'00'11'01, dy = field d of 0b11'01'00'00.
__device__ __forceinline__ void step_delta(uint32_t d, int &dx, int &dy) {
  dx = __builtin_amdgcn_sbfe(0x0D, d << 1, 2);
  dy = __builtin_amdgcn_sbfe(0xD0, d << 1, 2);
}

// Set the visited bit of lattice site c (row-major) in an LDS bitmap.
__device__ __forceinline__ void mark(uint32_t *bm, int c) { atomicOr(&bm[c >> 5], 1u << (c & 31)); }

// Walker bitmap modes: none, owned by this lane (plain read-modify-write),
// shared by the walker's segment lanes (global atomic or).
enum : int { WB_NONE = 0, WB_OWN = 1, WB_SHARED = 2 };

template <int WB>
__device__ __forceinline__ void mark_walker(uint32_t *wb, int c, bool active) {
  if (WB == WB_OWN && active) wb[c >> 5] |= 1u << (c & 31);
  if (WB == WB_SHARED && active) atomicOr(&wb[c >> 5], 1u << (c & 31));
}

// One move of a walker at unwrapped position (X, Y); marks the wrapped site.
// LDS: inactive lanes or into `spare` (a word past the bitmaps), so the
// mark needs no branch.
template <int GRID, bool LDS, int WB>
__device__ __forceinline__ void move1(uint32_t d, bool active, int &X, int &Y, uint32_t *bm,
                                      uint32_t *spare, uint32_t *wb) {
  int dx, dy;
  step_delta(d, dx, dy);
  X += dx;
  Y += dy;
  const int c = (Y & (GRID - 1)) * GRID + (X & (GRID - 1));
  if (LDS) {
    atomicOr(active ? &bm[c >> 5] : spare, 1u << (c & 31));
  } else {
    bm[c >> 5] |= 1u << (c & 31);
  }
  mark_walker<WB>(wb, c, active);
}

// Up to 16 moves from one 32-bit word (2 bits each, lowest first): moves
// g .. min(g + 16, steps) - 1.
template <int GRID, bool LDS, int WB = WB_NONE>
__device__ __forceinline__ void walk16(uint32_t word, uint32_t g, uint32_t steps, bool active,
                                       int &X, int &Y, uint32_t *bm, uint32_t *spare,
                                       uint32_t *wb = nullptr) {
  if (g + 16u <= steps) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      move1<GRID, LDS, WB>((word >> (2 * i)) & 3u, active, X, Y, bm, spare, wb);
  } else {
    for (uint32_t i = 0; g + i < steps; ++i)
      move1<GRID, LDS, WB>((word >> (2 * i)) & 3u, active, X, Y, bm, spare, wb);
  }
}

// (a << SH) + b and (a << SH) | b as one instruction each (the compiler
// splits the shift of a sign-extended field into two otherwise).
template <int SH>
__device__ __forceinline__ uint32_t lshl_add(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_lshl_add_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(SH), "v"(b));
  return r;
}
template <int SH>
__device__ __forceinline__ uint32_t lshl_or(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(SH), "v"(b));
  return r;
}

// The 16 moves of a word as sign-extended 2-bit dx and dy fields, so that a
// move's components are one bit-field extract each: d = 0 (+x) -> dx 01,
// 1 (-x) -> dx 11, 2 (+y) -> dy 01, 3 (-y) -> dy 11, 0 elsewhere.
__device__ __forceinline__ void split_moves(uint32_t word, uint32_t &DX, uint32_t &DY) {
  constexpr uint32_t M = 0x55555555u;
  const uint32_t L = word & M, H = (word >> 1) & M;  // low and high bit of each field
  DX = (H ^ M) | ((L & ~H) << 1);
  DY = H | ((H & L) << 1);
}

// Mark `mask` in the LDS word at byte address `addr`.
__device__ __forceinline__ void lds_or(uint32_t addr, uint32_t mask) {
  typedef __attribute__((address_space(3))) uint32_t lds_u32;
  __atomic_fetch_or((lds_u32 *)(uintptr_t)addr, mask, __ATOMIC_RELAXED);
}

// Up to 16 moves of every lane of a wavefront whose lanes are all walkers,
// on a GRID >= 32 torus, marking a row-major LDS bitmap (GRID / 32 words
// per row) at LDS byte address `base`. The walker keeps X and YB = Y *
// GRID / 8, the byte offset of its row (both unwrapped): a site's word is at
// base | (YB & rows) | ((X >> 3) & cols), its bit X & 31. Marks gather in
// the lane's pending word (paddr, pmask) while the walker stays in that
// word (an x move does, 31 times in 32) and reach LDS, as one or, when it
// leaves: about half the moves need no LDS operation.
// LDS byte address of the bitmap word holding site (X, Y) of the lean
// forms, from X and YB = Y * GRID / 8 (both unwrapped).
template <int GRID>
__device__ __forceinline__ uint32_t lean_word_addr(int X, int YB, uint32_t base) {
  constexpr int ROWB = GRID / 8;
  constexpr uint32_t ROWS = (uint32_t)(GRID * ROWB - 1) & ~(uint32_t)(ROWB - 1);
  constexpr uint32_t COLS = (uint32_t)(ROWB - 1) & ~3u;
  constexpr int LOG_COLW = GRID == 128 ? 2 : 1;
  const uint32_t row = ((uint32_t)YB & ROWS) | base;
  return COLS ? lshl_or<2>(__builtin_amdgcn_ubfe((uint32_t)X, 5, LOG_COLW), row) : row;
}

template <int GRID>
__device__ __forceinline__ void walk16_full(uint32_t word, uint32_t g, uint32_t steps, int &X,
                                           int &YB, uint32_t base, uint32_t &paddr,
                                           uint32_t &pmask) {
  static_assert(GRID >= 32, "a row of the bitmap is at least one word");
  constexpr int ROWB = GRID / 8;                           // bytes per row
  constexpr int LOG_ROWB = GRID == 32 ? 2 : GRID == 64 ? 3 : 4;
  constexpr uint32_t ROWS = (uint32_t)(GRID * ROWB - 1) & ~(uint32_t)(ROWB - 1);
  constexpr uint32_t COLS = (uint32_t)(ROWB - 1) & ~3u;
  constexpr int LOG_COLW = GRID == 128 ? 2 : 1;  // bits of the word index within a row
  uint32_t DX, DY;
  split_moves(word, DX, DY);
  auto move = [&](int i) {
    X += __builtin_amdgcn_sbfe((int)DX, 2 * i, 2);
    YB = (int)lshl_add<LOG_ROWB>((uint32_t)__builtin_amdgcn_sbfe((int)DY, 2 * i, 2), (uint32_t)YB);
    const uint32_t row = ((uint32_t)YB & ROWS) | base;
    const uint32_t addr =
        COLS ? lshl_or<2>(__builtin_amdgcn_ubfe((uint32_t)X, 5, LOG_COLW), row) : row;
    if (addr != paddr) {
      lds_or(paddr, pmask);
      pmask = 0u;
    }
    paddr = addr;
    pmask |= 1u << ((uint32_t)X & 31u);
  };
  if (g + 16u <= steps) {
#pragma unroll
    for (int i = 0; i < 16; ++i) move(i);
  } else {
    for (int i = 0; g + (uint32_t)i < steps; ++i) move(i);
  }
}

// The walk of a wavefront whose 64 lanes are all walkers, on Philox
// streams, in the lean form (GRID >= 32, no per-walker bitmaps); false when
// the form does not apply and nothing was done.
template <int GRID, bool PW>
__device__ __forceinline__ bool lean_walk(const RwArgs &a, uint64_t r, uint32_t w, uint32_t k0,
                                          uint32_t k1, uint32_t *bm, int &X, int &Y) {
  if constexpr (GRID >= 32 && !PW) {
    if (a.walkers != 64u) return false;
    if (r < a.n_reps) {
      constexpr int LOG_ROWB = GRID == 32 ? 2 : GRID == 64 ? 3 : 4;
      // the bitmap's LDS byte address (a multiple of its size, so the
      // site's offset can be or-ed into it)
      typedef __attribute__((address_space(3))) uint32_t lds_u32;
      const uint32_t base = (uint32_t)(uintptr_t)(lds_u32 *)bm;
      int YB = Y << LOG_ROWB;
      // the start site is the first pending mark
      const int c0 = Y * GRID + X;
      uint32_t paddr = base + 4u * ((uint32_t)c0 >> 5), pmask = 1u << (c0 & 31);
      for (uint32_t g = 0; g < a.steps; g += 64) {
        const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
        walk16_full<GRID>(b.x, g, a.steps, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.y, g + 16, a.steps, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.z, g + 32, a.steps, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.w, g + 48, a.steps, X, YB, base, paddr, pmask);
      }
      lds_or(paddr, pmask);
      Y = YB >> LOG_ROWB;  // arithmetic shift: YB is Y times a power of two
    }
    return true;
  } else {
    (void)a, (void)r, (void)w, (void)k0, (void)k1, (void)bm, (void)X, (void)Y;
    return false;
  }
}

// Pass 2 of the segmented walk in the lean form (every lane one segment of
// a walker, Philox, GRID >= 32, no per-walker bitmaps): the segment's moves
// from its start (X, Y), marking through the lane's pending word, which
// starts empty (the start site is the previous segment's last one, or the
// walker's start, marked apart); false when the form does not apply and
// nothing was done. `first`: the words of the segment's first 64 moves.
template <int GRID, int RNG, bool PW>
__device__ __forceinline__ bool lean_segment(const RwArgs &a, uint64_t r, uint32_t w, uint32_t k0,
                                             uint32_t k1, uint32_t t0, uint32_t t1,
                                             const uint32_t (&first)[4], uint32_t *bm, int X,
                                             int Y) {
  if constexpr (GRID >= 32 && !PW && RNG == RNG_PHILOX) {
    if (a.walkers != 64u) return false;
    constexpr int LOG_ROWB = GRID == 32 ? 2 : GRID == 64 ? 3 : 4;
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    const uint32_t base = (uint32_t)(uintptr_t)(lds_u32 *)bm;
    int YB = (int)((uint32_t)Y << LOG_ROWB);
    uint32_t paddr = lean_word_addr<GRID>(X, YB, base), pmask = 0u;
    if (t0 < t1) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        walk16_full<GRID>(first[j], t0 + 16u * j, t1, X, YB, base, paddr, pmask);
      for (uint32_t g = t0 + 64; g < t1; g += 64) {
        const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
        walk16_full<GRID>(b.x, g, t1, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.y, g + 16, t1, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.z, g + 32, t1, X, YB, base, paddr, pmask);
        walk16_full<GRID>(b.w, g + 48, t1, X, YB, base, paddr, pmask);
      }
    }
    lds_or(paddr, pmask);
    return true;
  } else {
    (void)a, (void)r, (void)w, (void)k0, (void)k1, (void)t0, (void)t1, (void)first, (void)bm,
        (void)X, (void)Y;
    return false;
  }
}

template <int GRID, int RNG, bool PW>
__global__ void rw_wave_kernel(RwArgs a) {
  constexpr int WORDS = GRID * GRID / 32;
  constexpr int WB = PW ? WB_OWN : WB_NONE;
  // aligned to the largest bitmap (128 x 128 bits), so that each
  // wavefront's bitmap address is a multiple of its size
  extern __shared__ __attribute__((aligned(2048))) uint32_t lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t *bm = lds + wave * WORDS;
  for (int i = lane; i < WORDS; i += 64) bm[i] = 0u;
  __syncthreads();

  const bool active = r < a.n_reps && (uint32_t)lane < a.walkers;
  const uint32_t w = (uint32_t)lane;
  const int x0 = (int)(((w % 8u) * (GRID / 8) + GRID / 16) % GRID);
  const int y0 = (int)(((w / 8u) * (GRID / 8) + GRID / 16) % GRID);
  int X = x0, Y = y0;
  uint32_t *spare = lds + (blockDim.x >> 6) * WORDS;
  if (active) mark(bm, y0 * GRID + x0);
  // this walker's own bitmap (global memory, owned by this lane)
  uint32_t *wb = nullptr;
  if (PW && active) {
    wb = a.walker_bitmaps + (r * a.walkers + w) * WORDS;
    for (int i = 0; i < WORDS; ++i) wb[i] = 0u;
    mark_walker<WB>(wb, y0 * GRID + x0, true);
  }

  if (RNG == RNG_TAUS88) {
    Taus t = taus_seed(TAG_RW, 0u, (uint32_t)(a.rep0 + r), k0, k1);
    taus_jump(t, a.taus_walk + (uint64_t)w * TAUS_COLS);  // to walker w's run
    for (uint32_t g = 0; g < a.steps; g += 16)
      walk16<GRID, true, WB>(taus_next(t), g, a.steps, active, X, Y, bm, spare, wb);
  } else if (lean_walk<GRID, PW>(a, r, w, k0, k1, bm, X, Y)) {
    // every lane a walker (or the whole wavefront idle): done in the lean form
  } else {
    for (uint32_t g = 0; g < a.steps; g += 64) {
      const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
      walk16<GRID, true, WB>(b.x, g, a.steps, active, X, Y, bm, spare, wb);
      walk16<GRID, true, WB>(b.y, g + 16, a.steps, active, X, Y, bm, spare, wb);
      walk16<GRID, true, WB>(b.z, g + 32, a.steps, active, X, Y, bm, spare, wb);
      walk16<GRID, true, WB>(b.w, g + 48, a.steps, active, X, Y, bm, spare, wb);
    }
  }
  __syncthreads();
  int cnt = 0;
  for (int i = lane; i < WORDS; i += 64) cnt += __popc(bm[i]);
  cnt = group_sum_i(cnt, 64);
  const int ux = X - x0, uy = Y - y0;
  const int sd = active ? ux * ux + uy * uy : 0;
  const int ssd = group_sum_i(sd, 64);
  int mine = 0;
  if (PW) {
    if (active)
      for (int i = 0; i < WORDS; ++i) mine += __popc(wb[i]);
    mine = group_sum_i(mine, 64);
  }
  if (lane == 0 && r < a.n_reps) {
    a.ssd[r] = ssd;
    a.distinct[r] = cnt;
    if (PW) a.walker_sites[r] = mine;
  }
}

// STRIDE = 1: one replication per lane. STRIDE = 64: one replication per
// wavefront with only its first lane working (the paper's WLP form, 63 of
// 64 lanes idle).
template <int GRID, int STRIDE, int RNG, bool PW>
__global__ void rw_simt_kernel(RwArgs a) {
  constexpr int WORDS = GRID * GRID / 32;
  constexpr int WB = PW ? WB_OWN : WB_NONE;
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t *bm = a.scratch_bitmaps + r * WORDS;
  for (int i = 0; i < WORDS; ++i) bm[i] = 0u;
  // one walker bitmap per replication, cleared for every walker
  uint32_t *wb = PW ? a.walker_bitmaps + r * WORDS : nullptr;
  int ssd = 0, mine = 0;
  Taus t;
  if (RNG == RNG_TAUS88) t = taus_seed(TAG_RW, 0u, (uint32_t)(a.rep0 + r), k0, k1);
  for (uint32_t w = 0; w < a.walkers; ++w) {
    const int x0 = (int)(((w % 8u) * (GRID / 8) + GRID / 16) % GRID);
    const int y0 = (int)(((w / 8u) * (GRID / 8) + GRID / 16) % GRID);
    int X = x0, Y = y0;
    bm[(y0 * GRID + x0) >> 5] |= 1u << ((y0 * GRID + x0) & 31);
    if (PW) {
      for (int i = 0; i < WORDS; ++i) wb[i] = 0u;
      mark_walker<WB>(wb, y0 * GRID + x0, true);
    }
    if (RNG == RNG_TAUS88) {
      for (uint32_t g = 0; g < a.steps; g += 16)
        walk16<GRID, false, WB>(taus_next(t), g, a.steps, true, X, Y, bm, nullptr, wb);
    } else {
      for (uint32_t g = 0; g < a.steps; g += 64) {
        const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
        walk16<GRID, false, WB>(b.x, g, a.steps, true, X, Y, bm, nullptr, wb);
        walk16<GRID, false, WB>(b.y, g + 16, a.steps, true, X, Y, bm, nullptr, wb);
        walk16<GRID, false, WB>(b.z, g + 32, a.steps, true, X, Y, bm, nullptr, wb);
        walk16<GRID, false, WB>(b.w, g + 48, a.steps, true, X, Y, bm, nullptr, wb);
      }
    }
    const int ux = X - x0, uy = Y - y0;
    ssd += ux * ux + uy * uy;
    if (PW)
      for (int i = 0; i < WORDS; ++i) mine += __popc(wb[i]);
  }
  int cnt = 0;
  for (int i = 0; i < WORDS; ++i) cnt += __popc(bm[i]);
  a.ssd[r] = ssd;
  a.distinct[r] = cnt;
  if (PW) a.walker_sites[r] = mine;
}

// Net displacement of moves g .. min(g + 16, steps) - 1 of one word.
__device__ __forceinline__ void word_displacement(uint32_t word, uint32_t g, uint32_t steps,
                                                  int &dx, int &dy) {
  const uint32_t n = g + 16u <= steps ? 16u : (g < steps ? steps - g : 0u);
  const uint32_t fields = n == 16u ? 0x55555555u : ((1u << (2u * n)) - 1u) & 0x55555555u;
  const uint32_t lo = word & fields, hi = (word >> 1) & fields;
  // d = 0: +x, 1: -x, 2: +y, 3: -y (hi:lo)
  dx += __popc(fields & ~hi & ~lo) - __popc(lo & ~hi);
  dy += __popc(hi & ~lo) - __popc(hi & lo);
}

// Sum of v over the workgroup (every thread gets it); `sh` holds one int per
// wavefront.
__device__ __forceinline__ int block_sum_i(int v, int *sh) {
  v = group_sum_i(v, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  int t = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// One workgroup per replication, 16 lanes per walker.
template <int GRID, int RNG, bool PW>
__global__ __launch_bounds__(1024) void rw_seg_kernel(RwArgs a, uint32_t seg) {
  constexpr int WORDS = GRID * GRID / 32;
  constexpr int WB = PW ? WB_SHARED : WB_NONE;
  // + the inactive lanes' spare word; aligned to the largest bitmap (128 x
  // 128 bits), so that the lean form can or a site's offset into its address
  __shared__ __attribute__((aligned(2048))) uint32_t bm[WORDS + 1];
  __shared__ int sh_red[16];
  const int tid = threadIdx.x;
  const uint32_t w = (uint32_t)tid >> 4, sgi = (uint32_t)tid & 15u;
  const uint64_t r = blockIdx.x;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  for (int i = tid; i < WORDS; i += blockDim.x) bm[i] = 0u;
  // the walker's own bitmap, shared by its 16 segment lanes (global memory)
  const bool active = w < a.walkers;
  uint32_t *wb = nullptr;
  if (PW && active) {
    wb = a.walker_bitmaps + (r * a.walkers + w) * WORDS;
    for (int i = (int)sgi; i < WORDS; i += 16) wb[i] = 0u;
  }
  __syncthreads();
  const uint32_t t0 = min(a.steps, sgi * seg), t1 = min(a.steps, t0 + seg);

  // pass 1: the segment's net displacement (seg is a multiple of 64 steps)
  Taus ts;
  if (RNG == RNG_TAUS88) {
    ts = taus_seed(TAG_RW, 0u, (uint32_t)(a.rep0 + r), k0, k1);
    // to walker w's run, then to this segment's start within it (w <= 63)
    taus_jump(ts, a.taus_walk + (uint64_t)w * TAUS_COLS);
    taus_jump(ts, a.taus_walk + (uint64_t)(TAUS_WALK_WALKERS + sgi) * TAUS_COLS);
  }
  // the first 64 moves' words are kept for pass 2 (for up to 1024 steps
  // that is the whole segment, and pass 2 draws nothing)
  uint32_t first[4] = {0u, 0u, 0u, 0u};
  Taus ts1 = ts;  // taus88: the state after those words
  int dx = 0, dy = 0;
  for (uint32_t g = t0; g < t1; g += 64) {
    uint32_t wd[4];
    if (RNG == RNG_TAUS88) {
#pragma unroll
      for (int j = 0; j < 4; ++j) wd[j] = g + 16u * j < t1 ? taus_next(ts) : 0u;
    } else {
      const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
      wd[0] = b.x;
      wd[1] = b.y;
      wd[2] = b.z;
      wd[3] = b.w;
    }
    if (g == t0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) first[j] = wd[j];
      ts1 = ts;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) word_displacement(wd[j], g + 16u * j, t1, dx, dy);
  }
  // inclusive scan over the walker's 16 segments, then this segment's start
  int sx = dx, sy = dy;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const int px = __shfl_up(sx, o, 16), py = __shfl_up(sy, o, 16);
    if ((int)sgi >= o) {
      sx += px;
      sy += py;
    }
  }
  const int x0 = (int)(((w % 8u) * (GRID / 8) + GRID / 16) % GRID);
  const int y0 = (int)(((w / 8u) * (GRID / 8) + GRID / 16) % GRID);
  if (active && sgi == 0) {
    mark(bm, y0 * GRID + x0);
    mark_walker<WB>(wb, y0 * GRID + x0, true);
  }
  // unwrapped position at the segment's start
  int X = x0 + (sx - dx), Y = y0 + (sy - dy);

  // pass 2: replay the segment's moves from its start
  if (lean_segment<GRID, RNG, PW>(a, r, w, k0, k1, t0, t1, first, bm, X, Y)) {
    // every lane a walker's segment: done in the lean form
  } else {
  if (t0 < t1) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      walk16<GRID, true, WB>(first[j], t0 + 16u * j, t1, active, X, Y, bm, &bm[WORDS], wb);
  }
  ts = ts1;
  for (uint32_t g = t0 + 64; g < t1; g += 64) {
    uint32_t wd[4];
    if (RNG == RNG_TAUS88) {
#pragma unroll
      for (int j = 0; j < 4; ++j) wd[j] = g + 16u * j < t1 ? taus_next(ts) : 0u;
    } else {
      const Block4 b = philox(g >> 6, w, (uint32_t)(a.rep0 + r), TAG_RW, k0, k1);
      wd[0] = b.x;
      wd[1] = b.y;
      wd[2] = b.z;
      wd[3] = b.w;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      walk16<GRID, true, WB>(wd[j], g + 16u * j, t1, active, X, Y, bm, &bm[WORDS], wb);
  }
  }
  __syncthreads();

  // outputs: the walkers' squared end displacements (last segment's lane
  // holds the walker's total) and the popcount of the union bitmap
  int mine = 0;
  if (PW && active) {
    // read the walker's words back through the atomic unit (where the other
    // segment lanes' ors were performed)
    for (int i = (int)sgi; i < WORDS; i += 16) mine += __popc(atomicOr(&wb[i], 0u));
  }
  const int sd = block_sum_i((active && sgi == 15) ? sx * sx + sy * sy : 0, sh_red);
  if (PW) mine = block_sum_i(mine, sh_red);
  int cnt = 0;
  for (int i = tid; i < WORDS; i += blockDim.x) cnt += __popc(bm[i]);
  cnt = block_sum_i(cnt, sh_red);
  if (tid == 0) {
    a.ssd[r] = sd;
    a.distinct[r] = cnt;
    if (PW) a.walker_sites[r] = mine;
  }
}

// Replications up to which the segmented form is used (measured for 64
// walkers x 1000 steps: 44 against 83 us at 1024 replications, 79 against
// 87 at 2048, 149 against 146 at 4096): below, the sequential form leaves
// the chip idle; above, its single pass over the moves is cheaper. On
// taus88 streams every segment lane first jumps to its place (two tables
// of 88 columns), so the sequential form wins earlier (64 x 1000: 39 against
// 55 us at 128 replications, 57 against 56 at 512, 90 against 56 at 1024,
// 148 against 78 at 2048).
constexpr uint64_t RW_SEG_MAX_REPS = 2048;
constexpr uint64_t RW_SEG_MAX_REPS_TAUS88 = 512;

template <int GRID>
hipError_t wave_launch(const RwArgs &a, uint32_t wg, hipStream_t s) {
  if (a.n_reps <= (a.rng == RNG_TAUS88 ? RW_SEG_MAX_REPS_TAUS88 : RW_SEG_MAX_REPS)) {
    // 16 lanes per walker; segments of whole Philox blocks (64 moves)
    const uint32_t threads = (16u * a.walkers + 63u) / 64u * 64u;
    const uint32_t seg = (a.steps + 16u * 64u - 1u) / (16u * 64u) * 64u;
    const dim3 g((uint32_t)a.n_reps), b(threads);
    const bool pw = a.walker_sites != nullptr;
    if (a.rng == RNG_TAUS88) {
      if (pw) hipLaunchKernelGGL((rw_seg_kernel<GRID, RNG_TAUS88, true>), g, b, 0, s, a, seg);
      else hipLaunchKernelGGL((rw_seg_kernel<GRID, RNG_TAUS88, false>), g, b, 0, s, a, seg);
    } else {
      if (pw) hipLaunchKernelGGL((rw_seg_kernel<GRID, RNG_PHILOX, true>), g, b, 0, s, a, seg);
      else hipLaunchKernelGGL((rw_seg_kernel<GRID, RNG_PHILOX, false>), g, b, 0, s, a, seg);
    }
    return hipGetLastError();
  }
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (a.n_reps + wpb - 1) / wpb;
  const size_t lds = ((size_t)wpb * (GRID * GRID / 32) + 1) * sizeof(uint32_t);  // + spare
  const dim3 g((uint32_t)blocks), b(wg);
  const bool pw = a.walker_sites != nullptr;
  if (a.rng == RNG_TAUS88) {
    if (pw) hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_TAUS88, true>), g, b, lds, s, a);
    else hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_TAUS88, false>), g, b, lds, s, a);
  } else {
    if (pw) hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_PHILOX, true>), g, b, lds, s, a);
    else hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_PHILOX, false>), g, b, lds, s, a);
  }
  return hipGetLastError();
}

template <int GRID>
hipError_t simt_launch(const RwArgs &a, bool one_lane, hipStream_t s) {
  const uint32_t wg = 64;
  const uint64_t threads = a.n_reps * (one_lane ? 64 : 1);
  const uint64_t blocks = (threads + wg - 1) / wg;
  const dim3 g((uint32_t)blocks), b(wg);
#define MRIP_SIMT(ST, RN, PW) hipLaunchKernelGGL((rw_simt_kernel<GRID, ST, RN, PW>), g, b, 0, s, a)
  const bool pw = a.walker_sites != nullptr;
  if (a.rng == RNG_TAUS88) {
    if (one_lane) { if (pw) MRIP_SIMT(64, RNG_TAUS88, true); else MRIP_SIMT(64, RNG_TAUS88, false); }
    else { if (pw) MRIP_SIMT(1, RNG_TAUS88, true); else MRIP_SIMT(1, RNG_TAUS88, false); }
  } else {
    if (one_lane) { if (pw) MRIP_SIMT(64, RNG_PHILOX, true); else MRIP_SIMT(64, RNG_PHILOX, false); }
    else { if (pw) MRIP_SIMT(1, RNG_PHILOX, true); else MRIP_SIMT(1, RNG_PHILOX, false); }
  }
#undef MRIP_SIMT
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rw_wave(const RwArgs &a, uint32_t wg, hipStream_t s) {
  switch (a.grid) {
    case 16: return wave_launch<16>(a, wg, s);
    case 32: return wave_launch<32>(a, wg, s);
    case 64: return wave_launch<64>(a, wg, s);
    case 128: return wave_launch<128>(a, wg, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rw_simt(const RwArgs &a, bool one_lane, hipStream_t s) {
  switch (a.grid) {
    case 16: return simt_launch<16>(a, one_lane, s);
    case 32: return simt_launch<32>(a, one_lane, s);
    case 64: return simt_launch<64>(a, one_lane, s);
    case 128: return simt_launch<128>(a, one_lane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mrip
