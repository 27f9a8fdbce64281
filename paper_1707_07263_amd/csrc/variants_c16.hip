#include "variants.hpp"

namespace mfft {

void add_variants_c16(void (*add)(const Variant&)) {
  add(make_variant<ROLE_ROW, 2, 16, 256, 0, __half2, 0>("r2p2w256_f16"));
  add(make_variant<ROLE_ROW, 4, 16, 256, 0, __half2, 0>("r4p4w256_f16"));
  add(make_variant<ROLE_ROW, 8, 16, 256, 0, __half2, 0>("r8p8w256_f16"));
  add(make_variant<ROLE_ROW, 16, 16, 256, 0, __half2, 0>("r16p16w256_f16"));
  add(make_variant<ROLE_ROW, 32, 16, 128, 0, __half2, 0>("r32p16w128_f16"));
  add(make_variant<ROLE_ROW, 64, 16, 64, 0, __half2, 0>("r64p16w64_f16"));
  add(make_variant<ROLE_ROW, 128, 16, 32, 0, __half2, 0>("r128p16w32_f16"));
  add(make_variant<ROLE_ROW, 256, 16, 16, 0, __half2, 0>("r256p16w16_f16"));
  add(make_variant<ROLE_ROW, 512, 16, 8, 0, __half2, 0>("r512p16w8_f16"));
  add(make_variant<ROLE_ROW, 1024, 16, 4, 0, __half2, 0>("r1024p16w4_f16"));
  add(make_variant<ROLE_ROW, 2048, 16, 2, 0, __half2, 0>("r2048p16w2_f16"));
  add(make_variant<ROLE_ROW, 4096, 16, 1, 0, __half2, 0>("r4096p16w1_f16"));
  add(make_variant<ROLE_ROW, 8192, 16, 1, 0, __half2, 0>("r8192p16w1_f16"));
  add(make_variant<ROLE_ROW, 16384, 16, 1, 0, __half2, 0>("r16384p16w1_f16"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 16, 0, __half2, 0>("a64p16w16_f16"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 16, 0, __half2, 0>("a128p16w16_f16"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, 0, __half2, 0>("a256p16w16_f16"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 0, __half2, 0>("a512p16w16_f16"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 16, 0, __half2, 0>("a1024p16w16_f16"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 8, 0, __half2, 0>("a2048p16w8_f16"));
  add(make_variant<ROLE_SPLIT_A, 4096, 16, 4, 0, __half2, 0>("a4096p16w4_f16"));
  add(make_variant<ROLE_COL, 2, 16, 16, 0, __half2, 0>("c2p2w16_f16"));
  add(make_variant<ROLE_COL, 4, 16, 16, 0, __half2, 0>("c4p4w16_f16"));
  add(make_variant<ROLE_COL, 8, 16, 16, 0, __half2, 0>("c8p8w16_f16"));
  add(make_variant<ROLE_COL, 16, 16, 16, 0, __half2, 0>("c16p16w16_f16"));
  add(make_variant<ROLE_COL, 32, 16, 16, 0, __half2, 0>("c32p16w16_f16"));
  add(make_variant<ROLE_COL, 64, 16, 16, 0, __half2, 0>("c64p16w16_f16"));
  add(make_variant<ROLE_COL, 128, 16, 16, 0, __half2, 0>("c128p16w16_f16"));
  add(make_variant<ROLE_COL, 256, 16, 16, 0, __half2, 0>("c256p16w16_f16"));
  add(make_variant<ROLE_COL, 512, 16, 16, 0, __half2, 0>("c512p16w16_f16"));
  add(make_variant<ROLE_COL, 1024, 16, 16, 0, __half2, 0>("c1024p16w16_f16"));
  add(make_variant<ROLE_COL, 2048, 16, 8, 0, __half2, 0>("c2048p16w8_f16"));
  add(make_variant<ROLE_COL, 4096, 16, 4, 0, __half2, 0>("c4096p16w4_f16"));
  add(make_variant<ROLE_COL, 8192, 16, 2, 0, __half2, 0>("c8192p16w2_f16"));
  add(make_variant<ROLE_COL, 16384, 16, 1, 0, __half2, 0>("c16384p16w1_f16"));
  add(make_variant<ROLE_ROW, 2, 16, 256, 0, c16bf, 0>("r2p2w256_bf16"));
  add(make_variant<ROLE_ROW, 4, 16, 256, 0, c16bf, 0>("r4p4w256_bf16"));
  add(make_variant<ROLE_ROW, 8, 16, 256, 0, c16bf, 0>("r8p8w256_bf16"));
  add(make_variant<ROLE_ROW, 16, 16, 256, 0, c16bf, 0>("r16p16w256_bf16"));
  add(make_variant<ROLE_ROW, 32, 16, 128, 0, c16bf, 0>("r32p16w128_bf16"));
  add(make_variant<ROLE_ROW, 64, 16, 64, 0, c16bf, 0>("r64p16w64_bf16"));
  add(make_variant<ROLE_ROW, 128, 16, 32, 0, c16bf, 0>("r128p16w32_bf16"));
  add(make_variant<ROLE_ROW, 256, 16, 16, 0, c16bf, 0>("r256p16w16_bf16"));
  add(make_variant<ROLE_ROW, 512, 16, 8, 0, c16bf, 0>("r512p16w8_bf16"));
  add(make_variant<ROLE_ROW, 1024, 16, 4, 0, c16bf, 0>("r1024p16w4_bf16"));
  add(make_variant<ROLE_ROW, 2048, 16, 2, 0, c16bf, 0>("r2048p16w2_bf16"));
  add(make_variant<ROLE_ROW, 4096, 16, 1, 0, c16bf, 0>("r4096p16w1_bf16"));
  add(make_variant<ROLE_ROW, 8192, 16, 1, 0, c16bf, 0>("r8192p16w1_bf16"));
  add(make_variant<ROLE_ROW, 16384, 16, 1, 0, c16bf, 0>("r16384p16w1_bf16"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 16, 0, c16bf, 0>("a64p16w16_bf16"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 16, 0, c16bf, 0>("a128p16w16_bf16"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, 0, c16bf, 0>("a256p16w16_bf16"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 0, c16bf, 0>("a512p16w16_bf16"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 16, 0, c16bf, 0>("a1024p16w16_bf16"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 8, 0, c16bf, 0>("a2048p16w8_bf16"));
  add(make_variant<ROLE_SPLIT_A, 4096, 16, 4, 0, c16bf, 0>("a4096p16w4_bf16"));
  add(make_variant<ROLE_COL, 2, 16, 16, 0, c16bf, 0>("c2p2w16_bf16"));
  add(make_variant<ROLE_COL, 4, 16, 16, 0, c16bf, 0>("c4p4w16_bf16"));
  add(make_variant<ROLE_COL, 8, 16, 16, 0, c16bf, 0>("c8p8w16_bf16"));
  add(make_variant<ROLE_COL, 16, 16, 16, 0, c16bf, 0>("c16p16w16_bf16"));
  add(make_variant<ROLE_COL, 32, 16, 16, 0, c16bf, 0>("c32p16w16_bf16"));
  add(make_variant<ROLE_COL, 64, 16, 16, 0, c16bf, 0>("c64p16w16_bf16"));
  add(make_variant<ROLE_COL, 128, 16, 16, 0, c16bf, 0>("c128p16w16_bf16"));
  add(make_variant<ROLE_COL, 256, 16, 16, 0, c16bf, 0>("c256p16w16_bf16"));
  add(make_variant<ROLE_COL, 512, 16, 16, 0, c16bf, 0>("c512p16w16_bf16"));
  add(make_variant<ROLE_COL, 1024, 16, 16, 0, c16bf, 0>("c1024p16w16_bf16"));
  add(make_variant<ROLE_COL, 2048, 16, 8, 0, c16bf, 0>("c2048p16w8_bf16"));
  add(make_variant<ROLE_COL, 4096, 16, 4, 0, c16bf, 0>("c4096p16w4_bf16"));
  add(make_variant<ROLE_COL, 8192, 16, 2, 0, c16bf, 0>("c8192p16w2_bf16"));
  add(make_variant<ROLE_COL, 16384, 16, 1, 0, c16bf, 0>("c16384p16w1_bf16"));
}

}  // namespace mfft
