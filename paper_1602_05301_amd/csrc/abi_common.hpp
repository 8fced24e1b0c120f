// Shared pieces of the C ABI implementation: thread-local error text and the
// opaque handle types.
#pragma once

#include <string>

#include "../../include/qbxfmm.h"
#include "planner.hpp"

struct qbx_plan_s {
    qbx::Plan pl;
};

namespace qbx {
void set_error(const std::string &msg);
qbx_status fail(qbx_status st, const std::string &msg);
// the calling thread's last message and a count of the messages it has set
std::string error_msg();
unsigned long long error_seq();
void fill_stats(const Plan &pl, qbx_stats *out);
}  // namespace qbx
