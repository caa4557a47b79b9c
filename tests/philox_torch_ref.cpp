// Independent Philox4x32-10 reference for the oracle's RNG pin: prints the
// block that PyTorch's header-only philox_engine produces for a counter and
// key given on the command line (8 hex words: c0 c1 c2 c3 k0 k1).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 7) return 2;
  uint32_t v[6];
  for (int i = 0; i < 6; ++i) v[i] = (uint32_t)strtoul(argv[i + 1], nullptr, 16);
  uint64_t seed = (uint64_t)v[4] | ((uint64_t)v[5] << 32);
  uint64_t subseq = (uint64_t)v[2] | ((uint64_t)v[3] << 32);
  uint64_t offset = (uint64_t)v[0] | ((uint64_t)v[1] << 32);
  at::philox_engine eng(seed, subseq, offset);
  for (int i = 0; i < 4; ++i) printf("%08x%s", eng(), i < 3 ? " " : "\n");
  return 0;
}
