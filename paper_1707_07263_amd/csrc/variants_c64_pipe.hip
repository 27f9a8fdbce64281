#include "variants.hpp"

namespace mfft {

void add_variants_c64_pipe(void (*add)(const Variant&)) {
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, 0, float2, 1>("a256p16w16q_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 32, 0, float2, 1>("a256p16w32q_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 8, 0, float2, 1>("a512p16w8q_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 0, float2, 1>("a512p16w16q_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 16, 0, float2, 1>("a512p32w16q_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 32, 0, float2, 1>("a512p32w32q_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 8, 0, float2, 1>("a1024p16w8q_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 8, 0, float2, 1>("a1024p32w8q_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 16, 0, float2, 1>("a1024p32w16q_c64"));
  add(make_variant<ROLE_COL, 256, 16, 16, 0, float2, 1>("c256p16w16q_c64"));
  add(make_variant<ROLE_COL, 256, 16, 32, 0, float2, 1>("c256p16w32q_c64"));
  add(make_variant<ROLE_COL, 256, 32, 32, 0, float2, 1>("c256p32w32q_c64"));
  add(make_variant<ROLE_COL, 512, 16, 8, 0, float2, 1>("c512p16w8q_c64"));
  add(make_variant<ROLE_COL, 512, 16, 16, 0, float2, 1>("c512p16w16q_c64"));
  add(make_variant<ROLE_COL, 512, 32, 16, 0, float2, 1>("c512p32w16q_c64"));
  add(make_variant<ROLE_COL, 512, 32, 32, 0, float2, 1>("c512p32w32q_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 8, 0, float2, 1>("c1024p16w8q_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 8, 0, float2, 1>("c1024p32w8q_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 16, 0, float2, 1>("c1024p32w16q_c64"));
  add(make_variant<ROLE_COL, 2048, 32, 8, 0, float2, 1>("c2048p32w8q_c64"));
  add(make_variant<ROLE_ROW, 1024, 16, 4, 0, float2, 1>("r1024p16w4q_c64"));
  add(make_variant<ROLE_ROW, 2048, 16, 2, 0, float2, 1>("r2048p16w2q_c64"));
  add(make_variant<ROLE_ROW, 2048, 16, 4, 0, float2, 1>("r2048p16w4q_c64"));
  add(make_variant<ROLE_ROW, 4096, 16, 1, 0, float2, 1>("r4096p16w1q_c64"));
  add(make_variant<ROLE_ROW, 4096, 16, 2, 0, float2, 1>("r4096p16w2q_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, 0, float2, 2>("a256p16w16q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 32, 0, float2, 2>("a256p16w32q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 8, 0, float2, 2>("a512p16w8q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 0, float2, 2>("a512p16w16q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 16, 0, float2, 2>("a512p32w16q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 32, 0, float2, 2>("a512p32w32q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 8, 0, float2, 2>("a1024p16w8q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 8, 0, float2, 2>("a1024p32w8q2_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 16, 0, float2, 2>("a1024p32w16q2_c64"));
  add(make_variant<ROLE_COL_TW, 2, 8, 8, 0, float2, 0>("t2p2w8_c64"));
  add(make_variant<ROLE_COL_TW, 2, 8, 16, 0, float2, 0>("t2p2w16_c64"));
  add(make_variant<ROLE_COL_TW, 2, 8, 32, 0, float2, 0>("t2p2w32_c64"));
  add(make_variant<ROLE_COL_TW, 2, 8, 64, 0, float2, 0>("t2p2w64_c64"));
  add(make_variant<ROLE_COL_TW, 4, 8, 8, 0, float2, 0>("t4p4w8_c64"));
  add(make_variant<ROLE_COL_TW, 4, 8, 16, 0, float2, 0>("t4p4w16_c64"));
  add(make_variant<ROLE_COL_TW, 4, 8, 32, 0, float2, 0>("t4p4w32_c64"));
  add(make_variant<ROLE_COL_TW, 4, 8, 64, 0, float2, 0>("t4p4w64_c64"));
  add(make_variant<ROLE_COL_TW, 8, 8, 8, 0, float2, 0>("t8p8w8_c64"));
  add(make_variant<ROLE_COL_TW, 8, 8, 16, 0, float2, 0>("t8p8w16_c64"));
  add(make_variant<ROLE_COL_TW, 8, 8, 32, 0, float2, 0>("t8p8w32_c64"));
  add(make_variant<ROLE_COL_TW, 8, 8, 64, 0, float2, 0>("t8p8w64_c64"));
  add(make_variant<ROLE_COL_TW, 16, 8, 8, 0, float2, 0>("t16p8w8_c64"));
  add(make_variant<ROLE_COL_TW, 16, 8, 16, 0, float2, 0>("t16p8w16_c64"));
  add(make_variant<ROLE_COL_TW, 16, 8, 32, 0, float2, 0>("t16p8w32_c64"));
  add(make_variant<ROLE_COL_TW, 16, 8, 64, 0, float2, 0>("t16p8w64_c64"));
  add(make_variant<ROLE_COL_TW, 16, 16, 8, 0, float2, 0>("t16p16w8_c64"));
  add(make_variant<ROLE_COL_TW, 16, 16, 16, 0, float2, 0>("t16p16w16_c64"));
  add(make_variant<ROLE_COL_TW, 16, 16, 32, 0, float2, 0>("t16p16w32_c64"));
  add(make_variant<ROLE_COL_TW, 16, 16, 64, 0, float2, 0>("t16p16w64_c64"));
  add(make_variant<ROLE_COL_TW, 32, 8, 8, 0, float2, 0>("t32p8w8_c64"));
  add(make_variant<ROLE_COL_TW, 32, 8, 16, 0, float2, 0>("t32p8w16_c64"));
  add(make_variant<ROLE_COL_TW, 32, 8, 32, 0, float2, 0>("t32p8w32_c64"));
  add(make_variant<ROLE_COL_TW, 32, 8, 64, 0, float2, 0>("t32p8w64_c64"));
  add(make_variant<ROLE_COL_TW, 32, 16, 8, 0, float2, 0>("t32p16w8_c64"));
  add(make_variant<ROLE_COL_TW, 32, 16, 16, 0, float2, 0>("t32p16w16_c64"));
  add(make_variant<ROLE_COL_TW, 32, 16, 32, 0, float2, 0>("t32p16w32_c64"));
  add(make_variant<ROLE_COL_TW, 32, 16, 64, 0, float2, 0>("t32p16w64_c64"));
  add(make_variant<ROLE_COL_TW, 64, 8, 8, 0, float2, 0>("t64p8w8_c64"));
  add(make_variant<ROLE_COL_TW, 64, 8, 16, 0, float2, 0>("t64p8w16_c64"));
  add(make_variant<ROLE_COL_TW, 64, 8, 32, 0, float2, 0>("t64p8w32_c64"));
  add(make_variant<ROLE_COL_TW, 64, 8, 64, 0, float2, 0>("t64p8w64_c64"));
  add(make_variant<ROLE_COL_TW, 64, 16, 16, 0, float2, 0>("t64p16w16_c64"));
  add(make_variant<ROLE_COL_TW, 64, 16, 32, 0, float2, 0>("t64p16w32_c64"));
  add(make_variant<ROLE_COL_TW, 64, 16, 64, 0, float2, 0>("t64p16w64_c64"));
  add(make_variant<ROLE_COL_TW, 128, 8, 8, 0, float2, 0>("t128p8w8_c64"));
  add(make_variant<ROLE_COL_TW, 128, 8, 16, 0, float2, 0>("t128p8w16_c64"));
  add(make_variant<ROLE_COL_TW, 128, 8, 32, 0, float2, 0>("t128p8w32_c64"));
  add(make_variant<ROLE_COL_TW, 128, 8, 64, 0, float2, 0>("t128p8w64_c64"));
  add(make_variant<ROLE_COL_TW, 128, 16, 8, 0, float2, 0>("t128p16w8_c64"));
  add(make_variant<ROLE_COL_TW, 128, 16, 16, 0, float2, 0>("t128p16w16_c64"));
  add(make_variant<ROLE_COL_TW, 128, 16, 32, 0, float2, 0>("t128p16w32_c64"));
  add(make_variant<ROLE_COL_TW, 128, 16, 64, 0, float2, 0>("t128p16w64_c64"));
}

}  // namespace mfft
