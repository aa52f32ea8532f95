// Second generator: L'Ecuyer's three-component Tausworthe generator taus88
// (Math. Comp. 65, 1996), the generator the paper's models draw from
// (section 5), with streams split by Random Spacing (section 5: each
// replication's stream starts from a random state).
//
// Component j keeps a k_j-bit state in the top bits of a word and advances
// s_j steps of the linear recurrence of the trinomial z^k + z^q + 1 at a
// time; the output is the xor of the three words after the step.
// (k, q, s) = (31, 13, 12), (29, 2, 4), (28, 3, 17).
//
// Random Spacing: the stream of (model, dp, replication) starts from words
// x, y, z of Philox block (model, dp, rep, 5) under the run's seed, each
// raised by 2, 8 or 16 when its k-bit part would be zero. Draw d of a
// replication is output d of its stream.
//
// Every step is linear over GF(2), so d steps are one 88-column matrix
// (per component, the images of the k state bits); lanes that start inside
// a stream jump there with tables of such matrices built on the host
// (taus_tables.cpp): table j advances 2^j outputs.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include "device.hpp"
#endif

namespace mrip {

constexpr int TAUS_K0 = 31, TAUS_Q0 = 13, TAUS_S0 = 12;
constexpr int TAUS_K1 = 29, TAUS_Q1 = 2, TAUS_S1 = 4;
constexpr int TAUS_K2 = 28, TAUS_Q2 = 3, TAUS_S2 = 17;
constexpr int TAUS_COLS = TAUS_K0 + TAUS_K1 + TAUS_K2;  // 88 words per table
constexpr int TAUS_POW2 = 64;                           // tables 2^0 .. 2^63
constexpr int TAUS_TABLES = TAUS_POW2;
constexpr uint32_t TAG_TAUS_SEED = 5;

// Host: fill `out` (TAUS_TABLES x TAUS_COLS words) with the jump tables.
void taus_build_tables(uint32_t *out);
// Host: the walk's jump tables for walks of `steps` moves, so that a lane
// reaches its place with one table per level instead of one per bit of the
// distance: table w (w < 64) advances to walker w's run (w ceil(steps/16)
// outputs), table 64 + s (s < 16) from a walker's run to its segment s
// (min(steps, s seg) / 16 outputs, seg the segmented form's moves per lane).
constexpr uint32_t TAUS_WALK_WALKERS = 64, TAUS_WALK_SEGMENTS = 16;
constexpr uint32_t TAUS_WALK_TABLES = TAUS_WALK_WALKERS + TAUS_WALK_SEGMENTS;
void taus_build_walk_tables(uint32_t steps, uint32_t *out);
// Host: the M/M/1 runs' jump tables for replications of `customers`
// customers. With L lanes per replication (16, 32, 64, 128 or 256) lane j
// takes the run of B = ceil(customers / L) customers starting at j B, 2 j B
// outputs into the stream; table i of L's group advances 2 B 2^i outputs,
// so a lane reaches its run with one table per set bit of j.
constexpr uint32_t TAUS_RUN_TABLES = 4 + 5 + 6 + 7 + 8;
constexpr uint32_t taus_run_base(uint32_t lanes) {
  return lanes == 16 ? 0u : lanes == 32 ? 4u : lanes == 64 ? 9u : lanes == 128 ? 15u : 22u;
}
void taus_build_run_tables(uint64_t customers, uint32_t *out);

#if defined(__HIPCC__)
struct Taus {
  uint32_t z0, z1, z2;
};

template <int K, int Q, int S>
__device__ __forceinline__ uint32_t taus_component(uint32_t z) {
  const uint32_t keep = 0xFFFFFFFFu << (32 - K);
  return ((z & keep) << S) ^ (((z << Q) ^ z) >> (K - S));
}

__device__ __forceinline__ uint32_t taus_next(Taus &t) {
  t.z0 = taus_component<TAUS_K0, TAUS_Q0, TAUS_S0>(t.z0);
  t.z1 = taus_component<TAUS_K1, TAUS_Q1, TAUS_S1>(t.z1);
  t.z2 = taus_component<TAUS_K2, TAUS_Q2, TAUS_S2>(t.z2);
  return t.z0 ^ t.z1 ^ t.z2;
}

// image of the k-bit state of z under one component's table columns
template <int K>
__device__ __forceinline__ uint32_t taus_apply(uint32_t z, const uint32_t *__restrict__ cols) {
  uint32_t acc = 0u;
  // a short unroll keeps one column and one mask live at a time
#pragma unroll 4
  for (int b = 0; b < K; ++b) {
    const uint32_t m = (uint32_t)((int32_t)(z << (K - 1 - b)) >> 31);  // bit 32-K+b
    acc ^= m & cols[b];
  }
  return acc;
}

__device__ __forceinline__ void taus_jump(Taus &t, const uint32_t *__restrict__ table) {
  t.z0 = taus_apply<TAUS_K0>(t.z0, table);
  t.z1 = taus_apply<TAUS_K1>(t.z1, table + TAUS_K0);
  t.z2 = taus_apply<TAUS_K2>(t.z2, table + TAUS_K0 + TAUS_K1);
}


// Random Spacing start state of the stream of (model, dp, rep).
__device__ __forceinline__ Taus taus_seed(uint32_t model, uint32_t dp, uint32_t rep, uint32_t k0,
                                          uint32_t k1) {
  const Block4 b = philox(model, dp, rep, TAG_TAUS_SEED, k0, k1);
  Taus t;
  t.z0 = b.x < 2u ? b.x + 2u : b.x;
  t.z1 = b.y < 8u ? b.y + 8u : b.y;
  t.z2 = b.z < 16u ? b.z + 16u : b.z;
  return t;
}

// Advance by d outputs with the power-of-two tables.
__device__ __forceinline__ void taus_skip(Taus &t, uint64_t d, const uint32_t *__restrict__ tables) {
  for (int j = 0; d != 0; ++j, d >>= 1)
    if (d & 1u) taus_jump(t, tables + (uint64_t)j * TAUS_COLS);
}
#endif

}  // namespace mrip
