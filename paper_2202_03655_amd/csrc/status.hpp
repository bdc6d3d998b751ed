// Error reporting shared by the C ABI translation units: the reason of the
// last failure is kept per thread and returned by hdf_last_error().
#pragma once
#include <string>

#include "../../include/hdf.h"

namespace hdf {
hdf_status set_error(hdf_status s, const std::string& msg);
void clear_error();
}  // namespace hdf
