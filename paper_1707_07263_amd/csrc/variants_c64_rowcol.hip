#include "variants.hpp"

namespace mfft {

void add_variants_c64_rowcol(void (*add)(const Variant&)) {
  add(make_rowcol_variant<256, 16, 4, 0, 1, float2>("f256p16w4q_c64"));
  add(make_rowcol_variant<512, 16, 4, 0, 1, float2>("f512p16w4q_c64"));
  add(make_rowcol_variant<1024, 32, 4, 0, 1, float2>("f1024p32w4q_c64"));
  add(make_rowcol_variant<2048, 32, 4, 0, 1, float2>("f2048p32w4q_c64"));
  add(make_rowcol_variant<4096, 32, 4, 1, 1, float2>("f4096p32w4qx_c64"));
  add(make_rowcol_variant<4096, 16, 4, 1, 1, float2>("f4096p16w4qx_c64"));
  add(make_rowcol_variant<4096, 32, 2, 1, 1, float2>("f4096p32w2qx_c64"));
  add(make_rowcol_variant<2048, 32, 2, 0, 1, float2>("f2048p32w2q_c64"));
  add(make_rowcol_variant<4096, 16, 4, 0, 2, float2>("f4096p16w4q_c64"));
  add(make_rowcol_variant<4096, 32, 4, 0, 2, float2>("f4096p32w4q_c64"));
  add(make_rowcol_variant<4096, 16, 2, 0, 2, float2>("f4096p16w2q_c64"));
  add(make_rowcol_variant<4096, 32, 2, 0, 2, float2>("f4096p32w2q_c64"));
}

}  // namespace mfft
