// Host-side helpers shared by the plan (plan.cpp) and the serving layer
// (server.cpp).
#pragma once

#include <string>

namespace prism {

// Record msg as the thread's last error (prism_last_error) and return code.
int set_error(int code, const std::string& msg);

}  // namespace prism
