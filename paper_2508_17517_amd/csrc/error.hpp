// Error type shared by the host code; no HIP dependency so the dense routines
// also build with a plain host compiler.
#pragma once

#include <stdexcept>
#include <string>

#include "airg.h"

namespace airg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

}  // namespace airg
