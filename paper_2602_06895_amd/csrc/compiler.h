// Host channel compiler: process description -> device tables.
#pragma once

#include <string>
#include <vector>

#include "json.h"
#include "tables.h"

namespace msx {

struct ChannelMeta {
    int process = 0;
    int dims = 0;
    int n_momenta = 0;  // n_final + 2
    int hadronic = 0;
    int nbins = 0;
};

struct Compiled {
    std::vector<ChannelTab> chans;
    std::vector<ProcessTab> procs;
    std::vector<ChannelMeta> meta;
};

// Compile a parsed description (one process object, or {"processes": [...]}).
bool compile_processes(const JValue& root, Compiled& out, std::string& err);

}  // namespace msx
