// Error handling shared by the C ABI entry points: exceptions become status
// codes and a thread-local message.
#pragma once

#include <new>
#include <string>

#include "common.hpp"

namespace fdm {

void set_error(const std::string& m);
void clear_error();

template <class F>
int guarded(F&& f) {
  try {
    clear_error();
    f();
    return FDM_OK;
  } catch (const Error& e) {
    set_error(e.what());
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return FDM_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    set_error(e.what());
    return FDM_ERR_STATE;
  }
}

// Fails with FDM_ERR_INVALID_ARG unless p is device (or managed) memory.
void check_device_ptr(const void* p, const char* what);

}  // namespace fdm
