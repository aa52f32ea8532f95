// Two independent Philox4x32-10 implementations used only to pin the
// oracle's Philox: PyTorch's header-only at::Philox4_32 and rocRAND's
// header-only philox4x32_10_engine. Both are driven through their public
// seed / subsequence / offset interface; neither is copied here.
#include <ATen/core/PhiloxRNGEngine.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>

extern "C" {

// key = (seed_lo, seed_hi); counter = (offset_lo, offset_hi, subseq_lo, subseq_hi).
void torch_philox_batch(uint64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t seed = (uint64_t)key[2 * i] | ((uint64_t)key[2 * i + 1] << 32);
    uint64_t offset = (uint64_t)ctr[4 * i] | ((uint64_t)ctr[4 * i + 1] << 32);
    uint64_t subseq = (uint64_t)ctr[4 * i + 2] | ((uint64_t)ctr[4 * i + 3] << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = eng();
  }
}

// rocRAND counts its offset in 32-bit outputs (4 per block); counter words
// 0..1 must stay below 2^62 for the offset to be representable.
void rocrand_philox_batch(uint64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t seed = (uint64_t)key[2 * i] | ((uint64_t)key[2 * i + 1] << 32);
    uint64_t blocks = (uint64_t)ctr[4 * i] | ((uint64_t)ctr[4 * i + 1] << 32);
    uint64_t subseq = (uint64_t)ctr[4 * i + 2] | ((uint64_t)ctr[4 * i + 3] << 32);
    rocrand_device::philox4x32_10_engine eng(seed, subseq, blocks * 4ull);
    for (int j = 0; j < 4; ++j) out[4 * i + j] = eng();
  }
}
}
