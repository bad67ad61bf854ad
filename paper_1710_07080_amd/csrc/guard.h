// Exception guard of the C entry points.
#pragma once

#include <exception>
#include <new>

#include "internal.h"

namespace isira {

// Runs an entry point's body and turns a C++ exception (a failed host allocation, say) into
// ISIRA_E_HOST, so that no exception crosses the C ABI.
template <typename F>
int guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(ISIRA_E_HOST, "host memory exhausted");
  } catch (const std::exception& e) {
    return set_error(ISIRA_E_HOST, e.what());
  } catch (...) {
    return set_error(ISIRA_E_HOST, "host-side failure");
  }
}

}  // namespace isira
