// Test shim: exposes the library's host path encoder (sx_encode.cpp, plain
// C++) through a C call, so the CPU suite can check it against the oracle's
// encoder without a GPU.  Test infrastructure only.
#include <cstring>
#include <string>

#include "sx_encode.h"

namespace {
sx::HostEncoding g_enc;
std::string g_err;
}  // namespace

extern "C" {
// Returns 0 on success, -1 on invalid input (message via shim_error).
int shim_encode(const sx_paths* paths, const sx_style* styles, uint32_t n_styles, uint32_t n_xforms) {
    return sx::encode_paths(*paths, styles, n_styles, n_xforms, g_enc, g_err) ? 0 : -1;
}
const char* shim_error() { return g_err.c_str(); }
uint32_t shim_n_tags() { return (uint32_t)g_enc.tags.size(); }
uint32_t shim_n_data() { return (uint32_t)g_enc.data.size(); }
uint32_t shim_n_styles() { return (uint32_t)g_enc.style_stream.size(); }
uint32_t shim_n_xforms() { return (uint32_t)g_enc.xform_stream.size(); }
uint32_t shim_n_paths() { return (uint32_t)g_enc.path_map.size(); }
void shim_copy(uint8_t* tags, float* data, uint32_t* style_stream, uint32_t* xform_stream, uint32_t* path_map) {
    if (!g_enc.tags.empty()) memcpy(tags, g_enc.tags.data(), g_enc.tags.size());
    if (!g_enc.data.empty()) memcpy(data, g_enc.data.data(), g_enc.data.size() * sizeof(float));
    if (!g_enc.style_stream.empty()) memcpy(style_stream, g_enc.style_stream.data(), g_enc.style_stream.size() * 4);
    if (!g_enc.xform_stream.empty()) memcpy(xform_stream, g_enc.xform_stream.data(), g_enc.xform_stream.size() * 4);
    if (!g_enc.path_map.empty()) memcpy(path_map, g_enc.path_map.data(), g_enc.path_map.size() * 4);
}
}
