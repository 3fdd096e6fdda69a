// Learned per-block format selection: the model hook of the planner.
#include "host.h"

namespace ffx {

bool learned_formats(const std::string& model_path, const std::vector<BlockStats>& blocks, std::vector<int32_t>& fmt) {
  (void)model_path;
  (void)blocks;
  (void)fmt;
  return false;  // no model: the planner falls back to the plain heuristic
}

}  // namespace ffx
