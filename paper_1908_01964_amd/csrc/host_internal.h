// Host-side helpers shared by the C ABI sources (not part of the public ABI).
#pragma once

#include <string>

#include "rcscm.h"

namespace rcscm {

// The host-side argument checks of rcscm_create / rcscm_create_batch: shapes,
// params, flags.  Returns OK or the status, with a message in *msg.
rcscm_status validate_args(int U, int I, const int* J, const int* M, const rcscm_params* p,
                           std::string* msg);

// Sets the message rcscm_last_error(NULL) returns (errors without a context).
void set_global_error(const std::string& msg);

}  // namespace rcscm
