// Exception barrier of the C ABI: every extern "C" entry point runs its body
// between FSI_ABI_TRY and FSI_ABI_CATCH, so no C++ exception (a failed host
// allocation inside a std::vector, std::map or std::string, or anything else)
// crosses the ABI. std::bad_alloc becomes FSI_ERR_OUT_OF_MEMORY, every other
// exception FSI_ERR_INTERNAL; both set the fsi_last_error() message.
#pragma once
#include <exception>
#include <new>

#include "../../include/fsi.h"

namespace fsi {
// Sets the thread-local fsi_last_error() message; never throws (a message
// that cannot be stored is dropped).
void record_error_noexcept(const char* msg) noexcept;
void record_error_noexcept2(const char* a, const char* b) noexcept;
// Test hook: true if the environment variable FSI_TEST_FAIL_ALLOC names this
// allocation site ("host": the plan's host tables; "device": the plan's
// device workspace). Lets tests force the out-of-memory paths.
bool test_fail_alloc(const char* site);
}  // namespace fsi

#define FSI_ABI_TRY try {
#define FSI_ABI_CATCH_RET(oom_ret, err_ret)                                          \
  }                                                                                  \
  catch (const std::bad_alloc&) {                                                    \
    ::fsi::record_error_noexcept("host allocation failed");                          \
    return oom_ret;                                                                  \
  }                                                                                  \
  catch (const std::exception& ex_) {                                                \
    ::fsi::record_error_noexcept2("internal error: ", ex_.what());                   \
    return err_ret;                                                                  \
  }                                                                                  \
  catch (...) {                                                                      \
    ::fsi::record_error_noexcept("internal error: unknown exception");               \
    return err_ret;                                                                  \
  }
#define FSI_ABI_CATCH FSI_ABI_CATCH_RET(FSI_ERR_OUT_OF_MEMORY, FSI_ERR_INTERNAL)
