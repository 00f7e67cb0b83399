#include "lp_device.h"
static void call_devlp(const void* fn, void* arg) {
  reinterpret_cast<void (*)(lpgpu::DevLP)>(const_cast<void*>(fn))(*static_cast<lpgpu::DevLP*>(arg));
}
extern const char* (*emu_kernel_name)(const void* fn);
static const char* kname(const void* fn) {
  using namespace lpgpu;
  if (fn == price_kernel(false)) return "k_price<false>";
  if (fn == price_kernel(true)) return "k_price<true>";
  if (fn == price_fin_kernel(false)) return "k_price_fin<false>";
  if (fn == price_fin_kernel(true)) return "k_price_fin<true>";
  if (fn == finish_kernel()) return "k_finish";
  if (fn == update_kernel_for_block(512)) return "k_update<512>";
  if (fn == update_kernel_for_block(1024)) return "k_update<1024>";
  if (fn == update_kernel_for_block(-512)) return "k_update_wide";
  {
    DevLP c{};
    c.cmode = 1;
    if (fn == update_kernel_for(c)) return "k_update_c";
  }
  if (fn == price32_kernel()) return "k_price32";
  if (fn == shortlist_kernel()) return "k_shortlist";
  return "struct-arg kernel";
}
struct EmuInit {
  EmuInit() {
    emu_call_struct = call_devlp;
    emu_struct_size = sizeof(lpgpu::DevLP);
    emu_kernel_name = kname;
  }
} emu_init;
