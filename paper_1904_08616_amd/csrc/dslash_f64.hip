// Template instances of the Dslash kernel for f64 storage.
#include "dslash_impl.h"

namespace dirac {

static const DslashEntry kTable[] = {
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStore, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStore, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStore, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStore, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiStore, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiStore, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiStore, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiStore, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStoreNorm, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStoreNorm, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStoreNorm, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, false, kEpiStoreNorm, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiSubNorm, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiSubNorm, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiSubNorm, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 18, true, kEpiSubNorm, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStore, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStore, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStore, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStore, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiStore, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiStore, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiStore, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiStore, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStoreNorm, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStoreNorm, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStoreNorm, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, false, kEpiStoreNorm, 4),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiSubNorm, 1),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiSubNorm, 2),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiSubNorm, 3),
    DIRAC_DSLASH_ENTRY(DIRAC_F64, DIRAC_F64, 12, true, kEpiSubNorm, 4),
};

const DslashEntry* dslash_table_f64(int* n) {
  *n = (int)(sizeof(kTable) / sizeof(kTable[0]));
  return kTable;
}

}  // namespace dirac
