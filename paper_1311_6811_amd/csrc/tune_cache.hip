// On-disk cache of the autotuners' choices (plans and batches): a flat JSON
// object of "key": tile pairs. Host code only.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <sys/stat.h>

#include "host_util.h"

namespace psfs {
namespace host {

std::string tune_cache_path()
{
    const char *p = std::getenv("PSFS_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char *home = std::getenv("HOME");
    return std::string(home && *home ? home : "/tmp") + "/.cache/psfs/autotune.json";
}

std::mutex &tune_cache_mutex()
{
    static std::mutex mu;
    return mu;
}

std::map<std::string, int> read_tune_cache(const std::string &path)
{
    std::map<std::string, int> m;
    std::ifstream in(path);
    if (!in) return m;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        const size_t colon = s.find(':', end);
        if (colon == std::string::npos) break;
        m[key] = std::atoi(s.c_str() + colon + 1);
        pos = s.find_first_of(",}", colon);
        if (pos == std::string::npos) break;
    }
    return m;
}

void write_tune_cache(const std::string &path, const std::map<std::string, int> &m)
{
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp";
    {
        std::ofstream out(tmp);
        out << "{\n";
        size_t i = 0;
        for (const auto &kv : m) out << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
        out << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

}  // namespace host
}  // namespace psfs
