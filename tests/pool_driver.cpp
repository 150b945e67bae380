// Test driver (host code, CPU only): runs the request server's first-fit
// allocator over an address range it never dereferences.  Reads commands from
// stdin -- "a BYTES" (allocate; prints the offset or -1), "r OFFSET BYTES"
// (release) -- and prints "USED PEAK_USED RANGES SIZE INDEX_OK" at the end.
#include <stdio.h>

#include "wrs_pool.h"

int main() {
    static char region[1];  // only its address is used
    char* base = region;
    size_t size = 0;
    if (scanf("%zu", &size) != 1) return 2;
    wrs::FirstFit ff;
    ff.reset(base, size);
    char op;
    while (scanf(" %c", &op) == 1) {
        if (op == 'a') {
            size_t b;
            if (scanf("%zu", &b) != 1) return 2;
            char* p = (char*)ff.alloc(b);
            printf("%lld\n", p ? (long long)(p - base) : -1LL);
        } else if (op == 'r') {
            size_t off, b;
            if (scanf("%zu %zu", &off, &b) != 2) return 2;
            ff.release(base + off, b);
        } else {
            return 2;
        }
    }
    printf("%zu %zu %zu %zu %d\n", ff.used(), ff.peak(), ff.free_ranges(), ff.size(), ff.index_consistent() ? 1 : 0);
    return 0;
}
