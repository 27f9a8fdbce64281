#include "variants.hpp"

namespace mfft {

void add_variants_c64_col(void (*add)(const Variant&)) {
  add(make_variant<ROLE_COL, 2, 8, 1, 0, float2, 0>("c2p2w1_c64"));
  add(make_variant<ROLE_COL, 2, 8, 2, 0, float2, 0>("c2p2w2_c64"));
  add(make_variant<ROLE_COL, 2, 8, 4, 0, float2, 0>("c2p2w4_c64"));
  add(make_variant<ROLE_COL, 2, 8, 8, 0, float2, 0>("c2p2w8_c64"));
  add(make_variant<ROLE_COL, 2, 8, 16, 0, float2, 0>("c2p2w16_c64"));
  add(make_variant<ROLE_COL, 2, 8, 32, 0, float2, 0>("c2p2w32_c64"));
  add(make_variant<ROLE_COL, 2, 8, 64, 0, float2, 0>("c2p2w64_c64"));
  add(make_variant<ROLE_COL, 4, 8, 1, 0, float2, 0>("c4p4w1_c64"));
  add(make_variant<ROLE_COL, 4, 8, 2, 0, float2, 0>("c4p4w2_c64"));
  add(make_variant<ROLE_COL, 4, 8, 4, 0, float2, 0>("c4p4w4_c64"));
  add(make_variant<ROLE_COL, 4, 8, 8, 0, float2, 0>("c4p4w8_c64"));
  add(make_variant<ROLE_COL, 4, 8, 16, 0, float2, 0>("c4p4w16_c64"));
  add(make_variant<ROLE_COL, 4, 8, 32, 0, float2, 0>("c4p4w32_c64"));
  add(make_variant<ROLE_COL, 4, 8, 64, 0, float2, 0>("c4p4w64_c64"));
  add(make_variant<ROLE_COL, 8, 8, 1, 0, float2, 0>("c8p8w1_c64"));
  add(make_variant<ROLE_COL, 8, 8, 2, 0, float2, 0>("c8p8w2_c64"));
  add(make_variant<ROLE_COL, 8, 8, 4, 0, float2, 0>("c8p8w4_c64"));
  add(make_variant<ROLE_COL, 8, 8, 8, 0, float2, 0>("c8p8w8_c64"));
  add(make_variant<ROLE_COL, 8, 8, 16, 0, float2, 0>("c8p8w16_c64"));
  add(make_variant<ROLE_COL, 8, 8, 32, 0, float2, 0>("c8p8w32_c64"));
  add(make_variant<ROLE_COL, 8, 8, 64, 0, float2, 0>("c8p8w64_c64"));
  add(make_variant<ROLE_COL, 16, 8, 1, 0, float2, 0>("c16p8w1_c64"));
  add(make_variant<ROLE_COL, 16, 8, 2, 0, float2, 0>("c16p8w2_c64"));
  add(make_variant<ROLE_COL, 16, 8, 4, 0, float2, 0>("c16p8w4_c64"));
  add(make_variant<ROLE_COL, 16, 8, 8, 0, float2, 0>("c16p8w8_c64"));
  add(make_variant<ROLE_COL, 16, 8, 16, 0, float2, 0>("c16p8w16_c64"));
  add(make_variant<ROLE_COL, 16, 8, 32, 0, float2, 0>("c16p8w32_c64"));
  add(make_variant<ROLE_COL, 16, 8, 64, 0, float2, 0>("c16p8w64_c64"));
  add(make_variant<ROLE_COL, 16, 16, 1, 0, float2, 0>("c16p16w1_c64"));
  add(make_variant<ROLE_COL, 16, 16, 2, 0, float2, 0>("c16p16w2_c64"));
  add(make_variant<ROLE_COL, 16, 16, 4, 0, float2, 0>("c16p16w4_c64"));
  add(make_variant<ROLE_COL, 16, 16, 8, 0, float2, 0>("c16p16w8_c64"));
  add(make_variant<ROLE_COL, 16, 16, 16, 0, float2, 0>("c16p16w16_c64"));
  add(make_variant<ROLE_COL, 16, 16, 32, 0, float2, 0>("c16p16w32_c64"));
  add(make_variant<ROLE_COL, 16, 16, 64, 0, float2, 0>("c16p16w64_c64"));
  add(make_variant<ROLE_COL, 32, 8, 1, 0, float2, 0>("c32p8w1_c64"));
  add(make_variant<ROLE_COL, 32, 8, 2, 0, float2, 0>("c32p8w2_c64"));
  add(make_variant<ROLE_COL, 32, 8, 4, 0, float2, 0>("c32p8w4_c64"));
  add(make_variant<ROLE_COL, 32, 8, 8, 0, float2, 0>("c32p8w8_c64"));
  add(make_variant<ROLE_COL, 32, 8, 16, 0, float2, 0>("c32p8w16_c64"));
  add(make_variant<ROLE_COL, 32, 8, 32, 0, float2, 0>("c32p8w32_c64"));
  add(make_variant<ROLE_COL, 32, 8, 64, 0, float2, 0>("c32p8w64_c64"));
  add(make_variant<ROLE_COL, 32, 16, 1, 0, float2, 0>("c32p16w1_c64"));
  add(make_variant<ROLE_COL, 32, 16, 2, 0, float2, 0>("c32p16w2_c64"));
  add(make_variant<ROLE_COL, 32, 16, 4, 0, float2, 0>("c32p16w4_c64"));
  add(make_variant<ROLE_COL, 32, 16, 8, 0, float2, 0>("c32p16w8_c64"));
  add(make_variant<ROLE_COL, 32, 16, 16, 0, float2, 0>("c32p16w16_c64"));
  add(make_variant<ROLE_COL, 32, 16, 32, 0, float2, 0>("c32p16w32_c64"));
  add(make_variant<ROLE_COL, 32, 16, 64, 0, float2, 0>("c32p16w64_c64"));
  add(make_variant<ROLE_COL, 64, 8, 8, 0, float2, 0>("c64p8w8_c64"));
  add(make_variant<ROLE_COL, 64, 8, 16, 0, float2, 0>("c64p8w16_c64"));
  add(make_variant<ROLE_COL, 64, 8, 32, 0, float2, 0>("c64p8w32_c64"));
  add(make_variant<ROLE_COL, 64, 8, 64, 0, float2, 0>("c64p8w64_c64"));
  add(make_variant<ROLE_COL, 64, 16, 16, 0, float2, 0>("c64p16w16_c64"));
  add(make_variant<ROLE_COL, 64, 16, 32, 0, float2, 0>("c64p16w32_c64"));
  add(make_variant<ROLE_COL, 64, 16, 64, 0, float2, 0>("c64p16w64_c64"));
  add(make_variant<ROLE_COL, 128, 8, 4, 0, float2, 0>("c128p8w4_c64"));
  add(make_variant<ROLE_COL, 128, 8, 8, 0, float2, 0>("c128p8w8_c64"));
  add(make_variant<ROLE_COL, 128, 8, 16, 0, float2, 0>("c128p8w16_c64"));
  add(make_variant<ROLE_COL, 128, 8, 32, 0, float2, 0>("c128p8w32_c64"));
  add(make_variant<ROLE_COL, 128, 8, 64, 0, float2, 0>("c128p8w64_c64"));
  add(make_variant<ROLE_COL, 128, 8, 64, 1, float2, 0>("c128p8w64x_c64"));
  add(make_variant<ROLE_COL, 128, 16, 8, 0, float2, 0>("c128p16w8_c64"));
  add(make_variant<ROLE_COL, 128, 16, 16, 0, float2, 0>("c128p16w16_c64"));
  add(make_variant<ROLE_COL, 128, 16, 32, 0, float2, 0>("c128p16w32_c64"));
  add(make_variant<ROLE_COL, 128, 16, 64, 0, float2, 0>("c128p16w64_c64"));
  add(make_variant<ROLE_COL, 128, 16, 64, 1, float2, 0>("c128p16w64x_c64"));
  add(make_variant<ROLE_COL, 256, 8, 2, 0, float2, 0>("c256p8w2_c64"));
  add(make_variant<ROLE_COL, 256, 8, 4, 0, float2, 0>("c256p8w4_c64"));
  add(make_variant<ROLE_COL, 256, 8, 8, 0, float2, 0>("c256p8w8_c64"));
  add(make_variant<ROLE_COL, 256, 8, 16, 0, float2, 0>("c256p8w16_c64"));
  add(make_variant<ROLE_COL, 256, 8, 32, 0, float2, 0>("c256p8w32_c64"));
  add(make_variant<ROLE_COL, 256, 8, 32, 1, float2, 0>("c256p8w32x_c64"));
  add(make_variant<ROLE_COL, 256, 16, 4, 0, float2, 0>("c256p16w4_c64"));
  add(make_variant<ROLE_COL, 256, 16, 8, 0, float2, 0>("c256p16w8_c64"));
  add(make_variant<ROLE_COL, 256, 16, 16, 0, float2, 0>("c256p16w16_c64"));
}

}  // namespace mfft
