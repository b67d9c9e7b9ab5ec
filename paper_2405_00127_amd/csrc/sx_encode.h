// Host path encoder (Section 8.2).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "strokex.h"

namespace sx {

struct HostEncoding {
    std::vector<uint8_t> tags;
    std::vector<float> data;             // x, y pairs
    std::vector<uint32_t> style_stream;  // caller style index per style entry
    std::vector<uint32_t> xform_stream;  // caller transform index per transform entry
    std::vector<uint32_t> path_map;      // encoded path -> input path
};

// styles: the caller's style table (n_styles entries); a path whose style
// has SX_STYLE_FILL gets every subpath closed.
bool encode_paths(const sx_paths& in, const sx_style* styles, uint32_t n_styles, uint32_t n_xforms,
                  HostEncoding& out, std::string& err);

}  // namespace sx
