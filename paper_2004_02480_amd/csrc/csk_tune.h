// csk_tune.h -- internal interface of the store of tuned launch choices.
#pragma once

#include <cstdarg>
#include <string>

namespace csk {

// A tuned choice: two integers whose meaning the kernel family fixes (grid
// and lanes per row; row tiles; plan variant) and the measured time.
struct TuneRec {
    int a, b;
    double us;
};

std::string device_arch();                 // the current device's architecture name
std::string tune_key(const char* fmt, ...);  // architecture-prefixed key
void tune_put(const std::string& key, const TuneRec& r);
bool tune_get(const std::string& key, TuneRec* out);
void tune_reset();
int tune_load_file(const char* path);      // entries read, or -1
bool tune_save_file(const char* path);
int tune_count();

}  // namespace csk
