#include "variants.hpp"

namespace mfft {

void add_variants_c64_row(void (*add)(const Variant&)) {
  add(make_variant<ROLE_ROW, 2, 8, 256, 0, float2, 0>("r2p2w256_c64"));
  add(make_variant<ROLE_ROW, 2, 8, 512, 0, float2, 0>("r2p2w512_c64"));
  add(make_variant<ROLE_ROW, 4, 8, 256, 0, float2, 0>("r4p4w256_c64"));
  add(make_variant<ROLE_ROW, 4, 8, 512, 0, float2, 0>("r4p4w512_c64"));
  add(make_variant<ROLE_ROW, 8, 8, 256, 0, float2, 0>("r8p8w256_c64"));
  add(make_variant<ROLE_ROW, 8, 8, 512, 0, float2, 0>("r8p8w512_c64"));
  add(make_variant<ROLE_ROW, 16, 8, 128, 0, float2, 0>("r16p8w128_c64"));
  add(make_variant<ROLE_ROW, 16, 8, 256, 0, float2, 0>("r16p8w256_c64"));
  add(make_variant<ROLE_ROW, 16, 16, 256, 0, float2, 0>("r16p16w256_c64"));
  add(make_variant<ROLE_ROW, 16, 16, 512, 0, float2, 0>("r16p16w512_c64"));
  add(make_variant<ROLE_ROW, 16, 16, 512, 1, float2, 0>("r16p16w512x_c64"));
  add(make_variant<ROLE_ROW, 32, 8, 64, 0, float2, 0>("r32p8w64_c64"));
  add(make_variant<ROLE_ROW, 32, 8, 128, 0, float2, 0>("r32p8w128_c64"));
  add(make_variant<ROLE_ROW, 32, 16, 128, 0, float2, 0>("r32p16w128_c64"));
  add(make_variant<ROLE_ROW, 32, 16, 256, 0, float2, 0>("r32p16w256_c64"));
  add(make_variant<ROLE_ROW, 32, 16, 256, 1, float2, 0>("r32p16w256x_c64"));
  add(make_variant<ROLE_ROW, 64, 8, 32, 0, float2, 0>("r64p8w32_c64"));
  add(make_variant<ROLE_ROW, 64, 8, 64, 0, float2, 0>("r64p8w64_c64"));
  add(make_variant<ROLE_ROW, 64, 16, 64, 0, float2, 0>("r64p16w64_c64"));
  add(make_variant<ROLE_ROW, 64, 16, 128, 0, float2, 0>("r64p16w128_c64"));
  add(make_variant<ROLE_ROW, 64, 16, 128, 1, float2, 0>("r64p16w128x_c64"));
  add(make_variant<ROLE_ROW, 128, 8, 16, 0, float2, 0>("r128p8w16_c64"));
  add(make_variant<ROLE_ROW, 128, 8, 32, 0, float2, 0>("r128p8w32_c64"));
  add(make_variant<ROLE_ROW, 128, 16, 32, 0, float2, 0>("r128p16w32_c64"));
  add(make_variant<ROLE_ROW, 128, 16, 64, 0, float2, 0>("r128p16w64_c64"));
  add(make_variant<ROLE_ROW, 128, 16, 64, 1, float2, 0>("r128p16w64x_c64"));
  add(make_variant<ROLE_ROW, 256, 8, 8, 0, float2, 0>("r256p8w8_c64"));
  add(make_variant<ROLE_ROW, 256, 8, 16, 0, float2, 0>("r256p8w16_c64"));
  add(make_variant<ROLE_ROW, 256, 16, 16, 0, float2, 0>("r256p16w16_c64"));
  add(make_variant<ROLE_ROW, 256, 16, 32, 0, float2, 0>("r256p16w32_c64"));
  add(make_variant<ROLE_ROW, 256, 16, 32, 1, float2, 0>("r256p16w32x_c64"));
  add(make_variant<ROLE_ROW, 512, 8, 4, 0, float2, 0>("r512p8w4_c64"));
  add(make_variant<ROLE_ROW, 512, 8, 8, 0, float2, 0>("r512p8w8_c64"));
  add(make_variant<ROLE_ROW, 512, 16, 8, 0, float2, 0>("r512p16w8_c64"));
  add(make_variant<ROLE_ROW, 512, 16, 16, 0, float2, 0>("r512p16w16_c64"));
  add(make_variant<ROLE_ROW, 512, 16, 16, 1, float2, 0>("r512p16w16x_c64"));
  add(make_variant<ROLE_ROW, 512, 32, 16, 0, float2, 0>("r512p32w16_c64"));
  add(make_variant<ROLE_ROW, 512, 32, 16, 1, float2, 0>("r512p32w16x_c64"));
  add(make_variant<ROLE_ROW, 512, 32, 32, 0, float2, 0>("r512p32w32_c64"));
  add(make_variant<ROLE_ROW, 512, 32, 32, 1, float2, 0>("r512p32w32x_c64"));
  add(make_variant<ROLE_ROW, 1024, 8, 2, 0, float2, 0>("r1024p8w2_c64"));
  add(make_variant<ROLE_ROW, 1024, 8, 4, 0, float2, 0>("r1024p8w4_c64"));
  add(make_variant<ROLE_ROW, 1024, 16, 4, 0, float2, 0>("r1024p16w4_c64"));
  add(make_variant<ROLE_ROW, 1024, 16, 8, 0, float2, 0>("r1024p16w8_c64"));
  add(make_variant<ROLE_ROW, 1024, 16, 8, 1, float2, 0>("r1024p16w8x_c64"));
  add(make_variant<ROLE_ROW, 1024, 32, 8, 0, float2, 0>("r1024p32w8_c64"));
  add(make_variant<ROLE_ROW, 1024, 32, 8, 1, float2, 0>("r1024p32w8x_c64"));
  add(make_variant<ROLE_ROW, 1024, 32, 16, 0, float2, 0>("r1024p32w16_c64"));
  add(make_variant<ROLE_ROW, 1024, 32, 16, 1, float2, 0>("r1024p32w16x_c64"));
  add(make_variant<ROLE_ROW, 2048, 8, 1, 0, float2, 0>("r2048p8w1_c64"));
  add(make_variant<ROLE_ROW, 2048, 8, 2, 0, float2, 0>("r2048p8w2_c64"));
  add(make_variant<ROLE_ROW, 2048, 16, 2, 0, float2, 0>("r2048p16w2_c64"));
  add(make_variant<ROLE_ROW, 2048, 16, 4, 0, float2, 0>("r2048p16w4_c64"));
  add(make_variant<ROLE_ROW, 2048, 16, 4, 1, float2, 0>("r2048p16w4x_c64"));
  add(make_variant<ROLE_ROW, 4096, 8, 1, 0, float2, 0>("r4096p8w1_c64"));
  add(make_variant<ROLE_ROW, 4096, 16, 1, 0, float2, 0>("r4096p16w1_c64"));
  add(make_variant<ROLE_ROW, 4096, 16, 2, 0, float2, 0>("r4096p16w2_c64"));
  add(make_variant<ROLE_ROW, 4096, 16, 2, 1, float2, 0>("r4096p16w2x_c64"));
  add(make_variant<ROLE_ROW, 8192, 8, 1, 0, float2, 0>("r8192p8w1_c64"));
  add(make_variant<ROLE_ROW, 8192, 8, 1, 1, float2, 0>("r8192p8w1x_c64"));
  add(make_variant<ROLE_ROW, 8192, 16, 1, 0, float2, 0>("r8192p16w1_c64"));
  add(make_variant<ROLE_ROW, 8192, 16, 1, 1, float2, 0>("r8192p16w1x_c64"));
  add(make_variant<ROLE_ROW, 16384, 16, 1, 0, float2, 0>("r16384p16w1_c64"));
  add(make_variant<ROLE_ROW, 16384, 16, 1, 1, float2, 0>("r16384p16w1x_c64"));
}

}  // namespace mfft
