#include "variants.hpp"

namespace mfft {

void add_variants_c64_col2(void (*add)(const Variant&)) {
  add(make_variant<ROLE_COL, 256, 16, 32, 0, float2, 0>("c256p16w32_c64"));
  add(make_variant<ROLE_COL, 256, 16, 32, 1, float2, 0>("c256p16w32x_c64"));
  add(make_variant<ROLE_COL, 256, 16, 64, 0, float2, 0>("c256p16w64_c64"));
  add(make_variant<ROLE_COL, 256, 16, 64, 1, float2, 0>("c256p16w64x_c64"));
  add(make_variant<ROLE_COL, 256, 32, 8, 0, float2, 0>("c256p32w8_c64"));
  add(make_variant<ROLE_COL, 256, 32, 16, 0, float2, 0>("c256p32w16_c64"));
  add(make_variant<ROLE_COL, 256, 32, 32, 0, float2, 0>("c256p32w32_c64"));
  add(make_variant<ROLE_COL, 256, 32, 32, 1, float2, 0>("c256p32w32x_c64"));
  add(make_variant<ROLE_COL, 256, 32, 64, 0, float2, 0>("c256p32w64_c64"));
  add(make_variant<ROLE_COL, 256, 32, 64, 1, float2, 0>("c256p32w64x_c64"));
  add(make_variant<ROLE_COL, 512, 8, 1, 0, float2, 0>("c512p8w1_c64"));
  add(make_variant<ROLE_COL, 512, 8, 2, 0, float2, 0>("c512p8w2_c64"));
  add(make_variant<ROLE_COL, 512, 8, 4, 0, float2, 0>("c512p8w4_c64"));
  add(make_variant<ROLE_COL, 512, 8, 8, 0, float2, 0>("c512p8w8_c64"));
  add(make_variant<ROLE_COL, 512, 8, 16, 0, float2, 0>("c512p8w16_c64"));
  add(make_variant<ROLE_COL, 512, 8, 16, 1, float2, 0>("c512p8w16x_c64"));
  add(make_variant<ROLE_COL, 512, 16, 2, 0, float2, 0>("c512p16w2_c64"));
  add(make_variant<ROLE_COL, 512, 16, 4, 0, float2, 0>("c512p16w4_c64"));
  add(make_variant<ROLE_COL, 512, 16, 8, 0, float2, 0>("c512p16w8_c64"));
  add(make_variant<ROLE_COL, 512, 16, 16, 0, float2, 0>("c512p16w16_c64"));
  add(make_variant<ROLE_COL, 512, 16, 16, 1, float2, 0>("c512p16w16x_c64"));
  add(make_variant<ROLE_COL, 512, 16, 32, 0, float2, 0>("c512p16w32_c64"));
  add(make_variant<ROLE_COL, 512, 16, 32, 1, float2, 0>("c512p16w32x_c64"));
  add(make_variant<ROLE_COL, 512, 32, 8, 0, float2, 0>("c512p32w8_c64"));
  add(make_variant<ROLE_COL, 512, 32, 16, 0, float2, 0>("c512p32w16_c64"));
  add(make_variant<ROLE_COL, 512, 32, 16, 1, float2, 0>("c512p32w16x_c64"));
  add(make_variant<ROLE_COL, 512, 32, 32, 0, float2, 0>("c512p32w32_c64"));
  add(make_variant<ROLE_COL, 512, 32, 32, 1, float2, 0>("c512p32w32x_c64"));
  add(make_variant<ROLE_COL, 512, 32, 64, 1, float2, 0>("c512p32w64x_c64"));
  add(make_variant<ROLE_COL, 1024, 8, 1, 0, float2, 0>("c1024p8w1_c64"));
  add(make_variant<ROLE_COL, 1024, 8, 2, 0, float2, 0>("c1024p8w2_c64"));
  add(make_variant<ROLE_COL, 1024, 8, 4, 0, float2, 0>("c1024p8w4_c64"));
  add(make_variant<ROLE_COL, 1024, 8, 8, 0, float2, 0>("c1024p8w8_c64"));
  add(make_variant<ROLE_COL, 1024, 8, 8, 1, float2, 0>("c1024p8w8x_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 1, 0, float2, 0>("c1024p16w1_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 2, 0, float2, 0>("c1024p16w2_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 4, 0, float2, 0>("c1024p16w4_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 8, 0, float2, 0>("c1024p16w8_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 8, 1, float2, 0>("c1024p16w8x_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 16, 0, float2, 0>("c1024p16w16_c64"));
  add(make_variant<ROLE_COL, 1024, 16, 16, 1, float2, 0>("c1024p16w16x_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 8, 0, float2, 0>("c1024p32w8_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 8, 1, float2, 0>("c1024p32w8x_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 16, 0, float2, 0>("c1024p32w16_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 16, 1, float2, 0>("c1024p32w16x_c64"));
  add(make_variant<ROLE_COL, 1024, 32, 32, 1, float2, 0>("c1024p32w32x_c64"));
  add(make_variant<ROLE_COL, 2048, 8, 1, 0, float2, 0>("c2048p8w1_c64"));
  add(make_variant<ROLE_COL, 2048, 8, 2, 0, float2, 0>("c2048p8w2_c64"));
  add(make_variant<ROLE_COL, 2048, 8, 4, 0, float2, 0>("c2048p8w4_c64"));
  add(make_variant<ROLE_COL, 2048, 8, 4, 1, float2, 0>("c2048p8w4x_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 1, 0, float2, 0>("c2048p16w1_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 2, 0, float2, 0>("c2048p16w2_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 4, 0, float2, 0>("c2048p16w4_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 4, 1, float2, 0>("c2048p16w4x_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 8, 0, float2, 0>("c2048p16w8_c64"));
  add(make_variant<ROLE_COL, 2048, 16, 8, 1, float2, 0>("c2048p16w8x_c64"));
  add(make_variant<ROLE_COL, 2048, 32, 8, 0, float2, 0>("c2048p32w8_c64"));
  add(make_variant<ROLE_COL, 2048, 32, 8, 1, float2, 0>("c2048p32w8x_c64"));
  add(make_variant<ROLE_COL, 2048, 32, 16, 1, float2, 0>("c2048p32w16x_c64"));
  add(make_variant<ROLE_COL, 4096, 8, 1, 0, float2, 0>("c4096p8w1_c64"));
  add(make_variant<ROLE_COL, 4096, 8, 2, 0, float2, 0>("c4096p8w2_c64"));
  add(make_variant<ROLE_COL, 4096, 8, 2, 1, float2, 0>("c4096p8w2x_c64"));
  add(make_variant<ROLE_COL, 4096, 16, 1, 0, float2, 0>("c4096p16w1_c64"));
  add(make_variant<ROLE_COL, 4096, 16, 2, 0, float2, 0>("c4096p16w2_c64"));
  add(make_variant<ROLE_COL, 4096, 16, 2, 1, float2, 0>("c4096p16w2x_c64"));
  add(make_variant<ROLE_COL, 4096, 16, 4, 0, float2, 0>("c4096p16w4_c64"));
  add(make_variant<ROLE_COL, 4096, 16, 4, 1, float2, 0>("c4096p16w4x_c64"));
  add(make_variant<ROLE_COL, 4096, 32, 8, 1, float2, 0>("c4096p32w8x_c64"));
  add(make_variant<ROLE_COL, 8192, 8, 1, 0, float2, 0>("c8192p8w1_c64"));
  add(make_variant<ROLE_COL, 8192, 8, 1, 1, float2, 0>("c8192p8w1x_c64"));
  add(make_variant<ROLE_COL, 8192, 16, 1, 0, float2, 0>("c8192p16w1_c64"));
  add(make_variant<ROLE_COL, 8192, 16, 1, 1, float2, 0>("c8192p16w1x_c64"));
  add(make_variant<ROLE_COL, 8192, 16, 2, 0, float2, 0>("c8192p16w2_c64"));
  add(make_variant<ROLE_COL, 8192, 16, 2, 1, float2, 0>("c8192p16w2x_c64"));
  add(make_variant<ROLE_COL, 16384, 16, 1, 0, float2, 0>("c16384p16w1_c64"));
  add(make_variant<ROLE_COL, 16384, 16, 1, 1, float2, 0>("c16384p16w1x_c64"));
}

}  // namespace mfft
