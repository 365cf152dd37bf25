// Host-side helpers shared by the translation units of the C ABI: the thread-local
// last-error message and launch checks.
#pragma once

#include "../../include/porta.h"

namespace porta {
namespace host {

// Records a printf-style message as the thread's last error and returns `code`.
int fail(int code, const char* fmt, ...);
// PORTA_EDEVICE with the HIP error text if the last launch failed, else PORTA_OK.
int check_launch(const char* what);
int validate_prec(int prec);

}  // namespace host
}  // namespace porta
