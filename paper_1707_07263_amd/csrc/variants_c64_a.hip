#include "variants.hpp"

namespace mfft {

void add_variants_c64_a(void (*add)(const Variant&)) {
  add(make_variant<ROLE_SPLIT_A, 64, 8, 8, float2>("a64p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 8, 16, float2>("a64p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 16, float2>("a64p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 8, 32, float2>("a64p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 64, 16, 32, float2>("a64p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 4, float2>("a128p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 8, float2>("a128p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 8, float2>("a128p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 16, float2>("a128p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 16, float2>("a128p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 8, 32, float2>("a128p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 128, 16, 32, float2>("a128p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 4, float2>("a256p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 4, float2>("a256p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 8, float2>("a256p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 8, float2>("a256p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 16, float2>("a256p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 16, float2>("a256p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 8, 32, float2>("a256p8w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 256, 16, 32, float2>("a256p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 4, float2>("a512p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 4, float2>("a512p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 8, float2>("a512p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 8, float2>("a512p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 8, 16, float2>("a512p8w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 16, float2>("a512p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 512, 16, 32, float2>("a512p16w32_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 8, 4, float2>("a1024p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 4, float2>("a1024p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 8, 8, float2>("a1024p8w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 8, float2>("a1024p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 1024, 16, 16, float2>("a1024p16w16_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 8, 4, float2>("a2048p8w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 4, float2>("a2048p16w4_c64"));
  add(make_variant<ROLE_SPLIT_A, 2048, 16, 8, float2>("a2048p16w8_c64"));
  add(make_variant<ROLE_SPLIT_A, 4096, 16, 4, float2>("a4096p16w4_c64"));
}

}  // namespace mfft
