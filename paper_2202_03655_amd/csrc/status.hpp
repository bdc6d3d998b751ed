// Shared by the C ABI translation units: the reason of the last failure, kept
// per thread and returned by hdf_last_error(), and the product-timing switch.
#pragma once
#include <string>

#include "../../include/hdf.h"

namespace hdf {
hdf_status set_error(hdf_status s, const std::string& msg);
void clear_error();
// Switch the HIP events around a factor's products on or off (hdf_info then
// reports no kernel times for them).  Products on many small factors use off.
void set_product_timing(hdf_handle h, bool on);
}  // namespace hdf
