// Buffers the sanitizer driver registers for the launcher stand-ins.
#pragma once
#include <cstddef>
void stub_register(const void* p, size_t bytes);
void stub_clear();
int stub_violations();
int stub_calls();
