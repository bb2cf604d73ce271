// On-disk cache of packed fast-form plans.  A plan file holds the packed op
// programs, the regenerated-block items and checkpoints and the build
// statistics of one (N, options) pair, so that a large plan (hours of host
// work at N = 4096) is built once and reloaded.
//
// File layout: magic "SHTPLAN\0", format version, the key string (every
// option that changes the factors, and the library's plan format version),
// payload length, 64-bit FNV-1a checksum of the payload, payload.  A file
// whose magic, version, length or checksum does not match is corrupt; a file
// whose key differs belongs to other options and is ignored.
#pragma once

#include <string>

#include "idbf_build.h"
#include "idbf_pack.h"
#include "sht.h"

namespace sht {
namespace idbf {

enum CacheStatus { kCacheOff = 0, kCacheHit = 1, kCacheMiss = 2, kCacheRebuilt = 3 };
const char *cache_status_name(int status);

// Key string of a plan of degree N with these options.
std::string cache_key(int N, const sht_plan_opts &o);
// File of that key under dir.
std::string cache_path(const std::string &dir, const std::string &key);

// Load: SHT_OK (hit), SHT_ERR_INVALID_ARG (no file, or another key's file),
// SHT_ERR_PLAN_CORRUPT (unreadable, truncated or checksum mismatch).
int cache_load(const std::string &path, const std::string &key, PackedPlan &pk, BuildStats &st);
// Store atomically (temporary file, then rename).  Returns SHT_OK or
// SHT_ERR_INVALID_ARG if the file cannot be written.
int cache_store(const std::string &path, const std::string &key, const PackedPlan &pk, const BuildStats &st);
// Check a file's header and checksum without keeping its contents.
int cache_verify(const std::string &path);

}  // namespace idbf
}  // namespace sht
