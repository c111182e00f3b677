// Host logging of the library (not device code).  With CURAST_LOG set in the environment to a
// value other than "0", the context set-up, each frame's plan, graph captures, autotuner results
// and every error are printed to stderr, one "[curast] ..." line each; unset, nothing is printed.
#pragma once
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace curast {

inline bool log_on()
{
    static const bool on = [] {
        const char* e = std::getenv("CURAST_LOG");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}

__attribute__((format(printf, 1, 2))) inline void log_line(const char* fmt, ...)
{
    if (!log_on()) return;
    std::va_list ap;
    va_start(ap, fmt);
    std::fputs("[curast] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

}  // namespace curast
