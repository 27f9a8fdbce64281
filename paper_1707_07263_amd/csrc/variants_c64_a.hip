#include "variants.hpp"

namespace mfft {

void add_variants_c64_a(void (*add)(const Variant&)) {
  add(make_variant<ROLE_SPLIT_A, 64, 8, 8, 0, float2, 0>("a64p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 8, 16, 0, float2, 0>("a64p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 8, 32, 0, float2, 0>("a64p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 8, 64, 0, float2, 0>("a64p8w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 16, 0, float2, 0>("a64p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 32, 0, float2, 0>("a64p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 64, 0, float2, 0>("a64p16w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 4, 0, float2, 0>("a128p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 8, 0, float2, 0>("a128p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 16, 0, float2, 0>("a128p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 32, 0, float2, 0>("a128p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 64, 0, float2, 0>("a128p8w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 64, 1, float2, 0>("a128p8w64x_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 8, 0, float2, 0>("a128p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 16, 0, float2, 0>("a128p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 32, 0, float2, 0>("a128p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 64, 0, float2, 0>("a128p16w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 64, 1, float2, 0>("a128p16w64x_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 4, 0, float2, 0>("a256p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 8, 0, float2, 0>("a256p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 16, 0, float2, 0>("a256p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 32, 0, float2, 0>("a256p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 32, 1, float2, 0>("a256p8w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 4, 0, float2, 0>("a256p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 8, 0, float2, 0>("a256p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, 0, float2, 0>("a256p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 32, 0, float2, 0>("a256p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 32, 1, float2, 0>("a256p16w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 64, 0, float2, 0>("a256p16w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 64, 1, float2, 0>("a256p16w64x_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 8, 0, float2, 0>("a256p32w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 16, 0, float2, 0>("a256p32w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 32, 0, float2, 0>("a256p32w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 32, 1, float2, 0>("a256p32w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 64, 0, float2, 0>("a256p32w64_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 32, 64, 1, float2, 0>("a256p32w64x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 4, 0, float2, 0>("a512p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 8, 0, float2, 0>("a512p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 16, 0, float2, 0>("a512p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 16, 1, float2, 0>("a512p8w16x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 4, 0, float2, 0>("a512p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 8, 0, float2, 0>("a512p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 0, float2, 0>("a512p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, 1, float2, 0>("a512p16w16x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 32, 0, float2, 0>("a512p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 32, 1, float2, 0>("a512p16w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 8, 0, float2, 0>("a512p32w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 16, 0, float2, 0>("a512p32w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 16, 1, float2, 0>("a512p32w16x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 32, 0, float2, 0>("a512p32w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 32, 1, float2, 0>("a512p32w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 32, 64, 1, float2, 0>("a512p32w64x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 8, 4, 0, float2, 0>("a1024p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 8, 8, 0, float2, 0>("a1024p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 8, 8, 1, float2, 0>("a1024p8w8x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 4, 0, float2, 0>("a1024p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 8, 0, float2, 0>("a1024p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 8, 1, float2, 0>("a1024p16w8x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 16, 0, float2, 0>("a1024p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 16, 1, float2, 0>("a1024p16w16x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 8, 0, float2, 0>("a1024p32w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 8, 1, float2, 0>("a1024p32w8x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 16, 0, float2, 0>("a1024p32w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 16, 1, float2, 0>("a1024p32w16x_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 32, 32, 1, float2, 0>("a1024p32w32x_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 8, 4, 0, float2, 0>("a2048p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 8, 4, 1, float2, 0>("a2048p8w4x_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 4, 0, float2, 0>("a2048p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 4, 1, float2, 0>("a2048p16w4x_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 8, 0, float2, 0>("a2048p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 8, 1, float2, 0>("a2048p16w8x_c64"));
  add(make_variant<ROLE_SPLIT_A, 4096, 16, 4, 0, float2, 0>("a4096p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 4096, 16, 4, 1, float2, 0>("a4096p16w4x_c64"));
}

}  // namespace mfft
