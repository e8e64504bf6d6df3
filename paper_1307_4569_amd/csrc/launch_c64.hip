// Kernel launchers instantiated for complex64 plans.
#include "launch.hpp"

namespace dgtns {
namespace host {

int forward_c64(const Plan& P, const void* f, int real_in, void* c, long long B, char* ws, const Layout& l,
                hipStream_t st) {
  return forward_impl<float2>(P, f, real_in, static_cast<float2*>(c), B, ws, l, st);
}

int forward_list_c64(const Plan& P, const void* const* f, int real_in, void* const* c, long long B, char* ws,
                     const Layout& l, hipStream_t st) {
  return forward_impl<float2>(P, nullptr, real_in, nullptr, B, ws, l, st, f, c);
}

int adjoint_c64(const Plan& P, const void* c, void* f, long long B, char* ws, const Layout& l, hipStream_t st) {
  return adjoint_impl<float2>(P, static_cast<const float2*>(c), static_cast<float2*>(f), B, ws, l, st);
}

int grad_c64(const Plan& P, const void* f, const void* gc, void* gg, long long B, char* ws, const Layout& l,
             hipStream_t st) {
  return grad_impl<float2>(P, static_cast<const float2*>(f), static_cast<const float2*>(gc), static_cast<float2*>(gg), B, ws, l,
                            st);
}

int set_window_c64(const Plan& P, const double2* g, char* ws, const Layout& l, hipStream_t st) {
  if (P.branch == kShearOla) {
    double2* gl = reinterpret_cast<double2*>(ws + l.ola_x);
    const int rc = ola_block_window(P, g, gl, st);
    if (rc) return rc;
    return set_window_c64(*P.inner, gl, ws + l.inner, ws_layout(*P.inner, DGTNS_OP_SET_WINDOW, 1), st);
  }
  return window_zak<float2>(P, g, mtab<float2>(P, P.off.zc), nullptr, ws, l, st);
}

}  // namespace host
}  // namespace dgtns
