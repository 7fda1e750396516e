// errors.hpp -- the library's error channel (amrv_last_error), shared by the
// forest entry points (api.cpp, which defines it) and the multigrid ones.
#pragma once

namespace amrv {

// records msg for amrv_last_error() and returns code
int set_error(int code, const char* msg);

}  // namespace amrv
