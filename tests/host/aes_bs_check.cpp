// Host check of the bitsliced AES-128 (paper_2606_09551_amd/csrc/fss_aes_bs.hpp):
// reads lines "k0 k1 ... k15 | p0 ... p15 | q0 ... q15" (hex bytes: a key and
// two plaintext blocks; the key must be the PRG key 00..0f for the fixed-key
// path) and prints the two ciphertexts, and "sbox" prints S(x) for x = 0..255
// through the bitsliced SubBytes.
#include <stdio.h>
#include <string.h>

#include "../../paper_2606_09551_amd/csrc/fss_aes_bs.hpp"
#include "../../paper_2606_09551_amd/csrc/fss_common.hpp"

using namespace fss;

static void words(const unsigned char* b, uint32_t (&w)[4]) {
  for (int c = 0; c < 4; ++c)
    w[c] = (uint32_t)b[4 * c] | ((uint32_t)b[4 * c + 1] << 8) | ((uint32_t)b[4 * c + 2] << 16) |
           ((uint32_t)b[4 * c + 3] << 24);
}

int main(int argc, char** argv) {
  static const bs::PrgPlanes rk = bs::make_prg_planes(kAes.prg_rk);
  if (argc > 1 && !strcmp(argv[1], "sbox")) {
    for (int base = 0; base < 256; base += 32) {
      uint32_t a[4], b[4], pl[8];
      unsigned char in[32];
      for (int j = 0; j < 32; ++j) in[j] = (unsigned char)(base + j);
      words(in, a);
      words(in + 16, b);
      bs::pack(a, b, pl);
      bs::sub_bytes(pl);
      bs::unpack(pl, a, b);
      for (int j = 0; j < 32; ++j) {
        const uint32_t w = j < 16 ? a[j / 4] : b[(j - 16) / 4];
        printf("%02x%s", (w >> (8 * (j % 4))) & 0xff, (base + j) % 16 == 15 ? "\n" : " ");
      }
    }
    return 0;
  }
  if (argc > 1 && !strcmp(argv[1], "roundtrip")) {
    uint32_t a[4] = {0x03020100u, 0x07060504u, 0x0b0a0908u, 0x0f0e0d0cu};
    uint32_t b[4] = {0xdeadbeefu, 0x01234567u, 0x89abcdefu, 0xfedcba98u}, pl[8], a2[4], b2[4];
    bs::pack(a, b, pl);
    bs::unpack(pl, a2, b2);
    for (int c = 0; c < 4; ++c)
      if (a2[c] != a[c] || b2[c] != b[c]) { printf("bad\n"); return 1; }
    printf("ok\n");
    return 0;
  }
  unsigned int k[16], p[16], q[16];
  while (scanf("%x %x %x %x %x %x %x %x %x %x %x %x %x %x %x %x |", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6],
               &k[7], &k[8], &k[9], &k[10], &k[11], &k[12], &k[13], &k[14], &k[15]) == 16) {
    for (int j = 0; j < 16; ++j) if (scanf("%x", &p[j]) != 1) return 2;
    if (scanf(" |") != 0) return 2;
    for (int j = 0; j < 16; ++j) if (scanf("%x", &q[j]) != 1) return 2;
    for (int j = 0; j < 16; ++j)
      if (k[j] != (unsigned)j) { printf("only the PRG key is supported\n"); return 3; }
    unsigned char pb[16], qb[16];
    for (int j = 0; j < 16; ++j) { pb[j] = (unsigned char)p[j]; qb[j] = (unsigned char)q[j]; }
    uint32_t a[4], b[4], pl[8];
    words(pb, a);
    words(qb, b);
    bs::pack(a, b, pl);
    bs::encrypt_pair(rk, pl);
    bs::unpack(pl, a, b);
    for (int j = 0; j < 16; ++j) printf("%02x", (a[j / 4] >> (8 * (j % 4))) & 0xff);
    printf(" ");
    for (int j = 0; j < 16; ++j) printf("%02x", (b[j / 4] >> (8 * (j % 4))) & 0xff);
    printf("\n");
  }
  return 0;
}
