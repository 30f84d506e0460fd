// Thread-local error message storage shared by the library's translation units.
#pragma once

namespace lodgs {

// Records msg as the calling thread's last error and returns code.
int set_error(int code, const char* msg);

}  // namespace lodgs
