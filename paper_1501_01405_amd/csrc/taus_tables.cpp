// Jump tables of the taus88 generator (see taus.hpp). One step of a
// component is linear over GF(2) in its k state bits, so d steps are a
// matrix; it is kept as the images of the k state bits (columns), and
// matrices compose column by column. Table j advances 2^j outputs (the j-th
// square of one step).
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "taus.hpp"

namespace mrip {

namespace {

struct Component {
  int k, q, s;
};
constexpr Component kComp[3] = {
    {TAUS_K0, TAUS_Q0, TAUS_S0}, {TAUS_K1, TAUS_Q1, TAUS_S1}, {TAUS_K2, TAUS_Q2, TAUS_S2}};

uint32_t step(uint32_t z, const Component &c) {
  const uint32_t keep = 0xFFFFFFFFu << (32 - c.k);
  return ((z & keep) << c.s) ^ (((z << c.q) ^ z) >> (c.k - c.s));
}

// a matrix of one component: col[b] = image of state bit 32-k+b
struct Mat {
  uint32_t col[32];
  int k;
};

uint32_t apply(const Mat &m, uint32_t z) {
  uint32_t acc = 0;
  for (int b = 0; b < m.k; ++b)
    if ((z >> (32 - m.k + b)) & 1u) acc ^= m.col[b];
  return acc;
}

// (a after b): first b, then a
Mat compose(const Mat &a, const Mat &b) {
  Mat r;
  r.k = a.k;
  for (int i = 0; i < b.k; ++i) r.col[i] = apply(a, b.col[i]);
  return r;
}

Mat one_step(const Component &c) {
  Mat m;
  m.k = c.k;
  for (int b = 0; b < c.k; ++b) m.col[b] = step(1u << (32 - c.k + b), c);
  return m;
}

void store(const Mat (&m)[3], uint32_t *table) {
  int o = 0;
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < m[c].k; ++b) table[o++] = m[c].col[b];
}

struct Pow2 {
  Mat m[TAUS_POW2][3];
  Pow2() {
    for (int c = 0; c < 3; ++c) m[0][c] = one_step(kComp[c]);
    for (int j = 1; j < TAUS_POW2; ++j)
      for (int c = 0; c < 3; ++c) m[j][c] = compose(m[j - 1][c], m[j - 1][c]);
  }
};

const Pow2 &pow2() {
  static const Pow2 p;
  return p;
}

// the table that advances d outputs (the product of the powers of two in d)
void store_jump(uint64_t d, uint32_t *out) {
  const Pow2 &p = pow2();
  Mat r[3];
  for (int c = 0; c < 3; ++c) {
    r[c].k = kComp[c].k;
    for (int b = 0; b < r[c].k; ++b) r[c].col[b] = 1u << (32 - r[c].k + b);  // identity
  }
  for (int j = 0; d != 0; ++j, d >>= 1)
    if (d & 1u)
      for (int c = 0; c < 3; ++c) r[c] = compose(p.m[j][c], r[c]);
  store(r, out);
}

}  // namespace

void taus_build_run_tables(uint64_t customers, uint32_t *out) {
  for (uint32_t lanes = 16; lanes <= 256; lanes *= 2) {
    const uint64_t run = (customers + lanes - 1) / lanes;  // customers per lane
    uint32_t *t = out + (size_t)taus_run_base(lanes) * TAUS_COLS;
    for (uint32_t i = 0; (1u << i) < lanes; ++i) store_jump(2 * run << i, t + (size_t)i * TAUS_COLS);
  }
}

void taus_build_tables(uint32_t *out) {
  const Pow2 &p = pow2();
  for (int j = 0; j < TAUS_POW2; ++j) store(p.m[j], out + (size_t)j * TAUS_COLS);
}

void taus_build_walk_tables(uint32_t steps, uint32_t *out) {
  const uint64_t per_walker = (steps + 15u) / 16u;                    // outputs of one walker
  const uint64_t seg = (steps + 16u * 64u - 1u) / (16u * 64u) * 64u;  // moves per segment
  for (uint32_t w = 0; w < TAUS_WALK_WALKERS; ++w)
    store_jump(w * per_walker, out + (size_t)w * TAUS_COLS);
  for (uint32_t s = 0; s < TAUS_WALK_SEGMENTS; ++s) {
    const uint64_t t0 = std::min<uint64_t>(steps, s * seg);
    store_jump(t0 / 16, out + (size_t)(TAUS_WALK_WALKERS + s) * TAUS_COLS);
  }
}

}  // namespace mrip
