// Helpers shared by the translation units that implement the C ABI.
#pragma once

#include <string>

#include "polydet.h"

namespace pd {

// Records msg as the calling thread's last error (polydet_last_error) and returns st.
polydet_status abi_fail(polydet_status st, const std::string& msg);

}  // namespace pd
