// Jump tables of the taus88 generator (see taus.hpp). One step of a
// component is linear over GF(2) in its k state bits, so d steps are a
// matrix; it is kept as the images of the k state bits (columns), and
// matrices compose column by column. Table j advances 2^j outputs (the j-th
// square of one step).
#include <stdint.h>

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

}  // namespace

void taus_build_tables(uint32_t *out) {
  Mat pow2[TAUS_POW2][3];
  for (int c = 0; c < 3; ++c) pow2[0][c] = one_step(kComp[c]);
  for (int j = 1; j < TAUS_POW2; ++j)
    for (int c = 0; c < 3; ++c) pow2[j][c] = compose(pow2[j - 1][c], pow2[j - 1][c]);
  for (int j = 0; j < TAUS_POW2; ++j) store(pow2[j], out + (size_t)j * TAUS_COLS);
}

}  // namespace mrip
