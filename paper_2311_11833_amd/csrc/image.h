// image.h -- the plan's device metadata as one host image (internal).
//
// Every index array the kernels read (permutations, fill patterns, level
// lists, update lists, step schedules, dense slot offsets) is laid out on the
// host in one int32 image, each part 256-byte aligned.  The caller provides
// device memory of image size and psp_plan_upload copies the image there; the
// pointers the kernels use are then set by relocation (field <- base + offset).
// The library itself never allocates device memory.
#pragma once

#include <cstdint>
#include <cstring>
#include <vector>

namespace psp {

struct PlanImage {
    std::vector<int32_t> words;
    struct Reloc {
        void* field;      // address of a `const T*` field inside the plan
        int64_t off;      // word offset of the part in the image
    };
    std::vector<Reloc> relocs;

    // Appends n words (zero-padded to a multiple of 64 words) and returns their offset.
    int64_t put(const int32_t* p, size_t n) {
        const int64_t off = (int64_t)words.size();
        words.insert(words.end(), p, p + n);
        words.resize((words.size() + 63) / 64 * 64, 0);
        return off;
    }
    int64_t put(const std::vector<int32_t>& v) { return put(v.data(), v.size()); }
    // Reserves n zero words.
    int64_t reserve(size_t n) {
        const int64_t off = (int64_t)words.size();
        words.resize((words.size() + n + 63) / 64 * 64, 0);
        return off;
    }
    template <class T>
    void bind(const T** field, int64_t off) { relocs.push_back({(void*)field, off}); }
    template <class T>
    void bind(T** field, int64_t off) { relocs.push_back({(void*)field, off}); }
    // Points every bound field at base + offset (base: the uploaded copy).
    void apply(const void* base) const {
        for (const Reloc& r : relocs) {
            const char* p = (const char*)base + 4 * r.off;
            std::memcpy(r.field, &p, sizeof(p));
        }
    }
    size_t bytes() const { return words.size() * sizeof(int32_t); }
};

}  // namespace psp
