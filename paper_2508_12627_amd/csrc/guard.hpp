// Every extern "C" entry point runs its body inside this guard, so that no
// C++ exception crosses the ABI: a host allocation failure becomes
// USTAT_E_NOMEM and any other exception USTAT_E_INVALID, each with a
// thread-local message (ustat_last_error).
#pragma once

#include <exception>
#include <new>
#include <string>

namespace ustat {
void set_last_error(const std::string &msg);
}

#define USTAT_GUARD_BEGIN try {
#define USTAT_GUARD_END                                                          \
    }                                                                            \
    catch (const std::bad_alloc &) {                                             \
        ::ustat::set_last_error("host allocation failed");                       \
        return USTAT_E_NOMEM;                                                    \
    }                                                                            \
    catch (const std::exception &ex_) {                                          \
        ::ustat::set_last_error(std::string("host exception: ") + ex_.what());   \
        return USTAT_E_INVALID;                                                  \
    }                                                                            \
    catch (...) {                                                                \
        ::ustat::set_last_error("unexpected host exception");                    \
        return USTAT_E_INVALID;                                                  \
    }
